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
//
// CNOT ladder.  CNOT(q -> q+1) for q = 0..NQ-2 in order maps basis index k
// to its prefix parity: bit j of pi(k) is the parity of bits 0..j of k.
// After a ladder the registers are left in the ladder frame (stored index k
// holds the true amplitude of pi(k)) and the next relayout writes each
// amplitude to LDS slot pi(k), which returns to the true frame at no cost.
// In the ladder frame, RY on true qubit q pairs k with
// pi^-1(pi(k) ^ 2^q) = k ^ 2^q ^ 2^{q+1} (k ^ 2^q for the last qubit), and
// the member with bit q clear is the true |0> member iff bits 0..q-1 of k
// have even parity (else the pair turns by -angle).  Both bits are register
// bits for every qubit of the HI layout and for qubits 0..RB-2 of LO; qubit
// RB-1 of LO pairs register bit RB-1 with lane bit 0, a DPP lane swap.
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
    // global basis index of (lane, r); bit NQ is the half.  The lane and
    // register parts occupy disjoint bits: g = glane(lane) | greg(r).
    __device__ static __forceinline__ int glane(int lane) {
        return HI ? ((lane & 31) | ((lane >> 5) << NQ)) : (((lane & 31) << RB) | ((lane >> 5) << NQ));
    }
    __host__ __device__ static constexpr int greg(int r) { return HI ? (r << 5) : r; }
    __device__ static __forceinline__ int g(int lane, int r) { return glane(lane) | greg(r); }
};

// LDS slot of basis index g: one pad amplitude every 32.
__device__ __forceinline__ int pad_slot(int g) { return g + (g >> 5); }

// pad_slot(Lay<NQ, HI>::g(lane, r)).  With SPLIT, as a per-lane base plus a
// per-register offset: the lane and register parts of g occupy disjoint
// bits, and so do their parts above bit 5, so g + (g >> 5) is the sum of the
// same expression over each part; with r known at compile time the offset
// becomes the LDS instruction's immediate and the address costs no
// instruction per register.  The float32 kernels take the split (fewer
// instructions and registers, one more wavefront per SIMD); the float64
// kernels measured faster with the combined index and keep it.
template <int NQ, bool HI, bool SPLIT>
struct SlotMap {
    int lg, base;
    __device__ __forceinline__ explicit SlotMap(int lane)
        : lg(Lay<NQ, HI>::glane(lane)), base(pad_slot(Lay<NQ, HI>::glane(lane))) {}
    __host__ __device__ static constexpr int roff(int r) {
        return Lay<NQ, HI>::greg(r) + (Lay<NQ, HI>::greg(r) >> 5);
    }
    __device__ __forceinline__ int operator()(int r) const {
        if constexpr (SPLIT)
            return base + roff(r);
        else
            return pad_slot(lg | Lay<NQ, HI>::greg(r));
    }
};

template <typename T>
constexpr bool kSplitSlots = sizeof(T) == 4;

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
    T mtp = -tp, mtn = tp, spp = sp, spn = -sp;
    // float64: with the four factors held as opaque registers every shear
    // is an in-place v_fmac_f64 instead of a v_fma_f64 with a negated
    // operand into a second register (5.7 % faster evaluation at n = 10 with
    // the CZ ladder; the float32 kernels and the ladder routine below were
    // measured slower with it)
    if constexpr (sizeof(T) == 8) asm volatile("" : "+v"(mtp), "+v"(mtn), "+v"(spp), "+v"(spn));
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
    const SlotMap<NQ, FROM_HI, kSplitSlots<T>> from(lane);
#pragma unroll
    for (int r = 0; r < R; ++r) S[from(r)] = {re[r], im[r]};
    __syncthreads();
    const SlotMap<NQ, !FROM_HI, kSplitSlots<T>> to(lane);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const cplx<T> v = S[to(r)];
        re[r] = v.re;
        im[r] = v.im;
    }
    __syncthreads();
}

// Planar LDS image: one component at a time in 2^(NQ+1) (+ pad) values.
// A float64 state takes 16 B per amplitude, so the interleaved image (33 KB
// at NQ = 10) holds a CU to four wavefronts; the planar one (17 KB) moves
// the real parts and then the imaginary parts through half the space.
template <typename T, int NQ, bool FROM_HI>
__device__ __forceinline__ void relayout_plane(T* x, T* P, int lane) {
    constexpr int R = Lay<NQ, FROM_HI>::R;
    const SlotMap<NQ, FROM_HI, kSplitSlots<T>> from(lane);
#pragma unroll
    for (int r = 0; r < R; ++r) P[from(r)] = x[r];
    __syncthreads();
    const SlotMap<NQ, !FROM_HI, kSplitSlots<T>> to(lane);
#pragma unroll
    for (int r = 0; r < R; ++r) x[r] = P[to(r)];
    __syncthreads();
}

template <typename T, int NQ, bool FROM_HI>
__device__ __forceinline__ void relayout(T* re, T* im, T* P, int lane) {
    relayout_plane<T, NQ, FROM_HI>(re, P, lane);
    relayout_plane<T, NQ, FROM_HI>(im, P, lane);
}

// ---------------------------------------------------------------- CNOT ladder

// pi on the NQ system bits of g (bit NQ, the half, is kept); linear over
// GF(2), so pi(glane ^ greg) = pi(glane) ^ pi(greg).
template <int NQ>
__host__ __device__ constexpr int ladder_perm(int g) {
    static_assert(NQ <= 16, "prefix parity over at most 16 bits");
    constexpr int M = (1 << NQ) - 1;
    int y = g & M;
    y ^= y << 1;
    y ^= y << 2;
    y ^= y << 4;
    y ^= y << 8;
    return (y & M) | (g & ~M);
}

__host__ __device__ constexpr bool odd_bits(int v) {
    bool p = false;
    for (; v; v &= v - 1) p = !p;
    return p;
}

// RY on true qubit Q with the registers in the ladder frame (both bits of
// the stored pair in registers).
template <typename T, int NQ, bool HI, int Q>
__device__ __forceinline__ void ry_reg_ladder(T* re, T* im, int lane, T t, T s) {
    using Ly = Lay<NQ, HI>;
    constexpr int R = Ly::R;
    constexpr int j = Ly::reg(Q);
    constexpr int jp = Q + 1 < NQ ? Ly::reg(Q + 1) : -1;
    static_assert(j >= 0 && (Q + 1 == NQ || jp >= 0), "pair not in registers");
    constexpr int mask = (1 << j) | (jp >= 0 ? (1 << jp) : 0);
    // register bits that hold the qubits below Q (lane bits hold the rest in HI)
    constexpr int low = HI ? ((1 << (Q - 5)) - 1) : ((1 << Q) - 1);
    T tp = t, sp = s;
    if constexpr (HI) {
        if (__popc((unsigned)(lane & 31)) & 1) {
            tp = -t;
            sp = -s;
        }
    }
    const T mtp = -tp, mtn = tp, spp = sp, spn = -sp;
#pragma unroll
    for (int r0 = 0; r0 < R; ++r0) {
        if (r0 & (1 << j)) continue;
        const int r1 = r0 ^ mask;
        const bool neg = odd_bits(r0 & low);
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

template <typename T, int NQ, bool HI, int Q, int QEND>
__device__ __forceinline__ void ry_range_ladder(T* re, T* im, int lane, const T* trig, int kbase) {
    if constexpr (Q < QEND) {
        ry_reg_ladder<T, NQ, HI, Q>(re, im, lane, trig[2 * (kbase + Q)], trig[2 * (kbase + Q) + 1]);
        ry_range_ladder<T, NQ, HI, Q + 1, QEND>(re, im, lane, trig, kbase);
    }
}

// Value held by lane ^ 1 (DPP quad permutation [1, 0, 3, 2]).
__device__ __forceinline__ float lane_xor1(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xB1, 0xF, 0xF, false));
}

__device__ __forceinline__ double lane_xor1(double x) {
    const long long u = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)u, 0xB1, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), 0xB1, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// RY on true qubit RB-1 in layout LO, ladder frame: the stored partner of
// (lane, r) is (lane ^ 1, r ^ 2^(RB-1)); bits 0..RB-1 of k are the register
// bits, so the amplitude is the true |1> member iff r has odd parity.
// Direct form: x' = cos(phi) x -+ sin(phi) p.
template <typename T, int NQ>
__device__ __forceinline__ void ry_lane_ladder_lo(T* re, T* im, T t, T s) {
    using Ly = Lay<NQ, false>;
    constexpr int R = Ly::R, j = Ly::RB - 1;
    static_assert(Ly::lanebit(Ly::RB) == 0, "qubit RB must sit in lane bit 0");
    const T c = fmat(-t, s, (T)1);  // cos(phi) = 1 - tan(phi/2) sin(phi)
#pragma unroll
    for (int r0 = 0; r0 < R; ++r0) {
        if (r0 & (1 << j)) continue;
        const int r1 = r0 | (1 << j);
        const T p0r = lane_xor1(re[r1]), p0i = lane_xor1(im[r1]);  // partner of r0
        const T p1r = lane_xor1(re[r0]), p1i = lane_xor1(im[r0]);  // partner of r1
        const T s0 = odd_bits(r0) ? s : -s, s1 = odd_bits(r1) ? s : -s;
        re[r0] = fmat(s0, p0r, c * re[r0]);
        im[r0] = fmat(s0, p0i, c * im[r0]);
        re[r1] = fmat(s1, p1r, c * re[r1]);
        im[r1] = fmat(s1, p1i, c * im[r1]);
    }
}

// pi^-1(m) = m ^ (m << 1) on the system bits.
template <int NQ>
__host__ __device__ constexpr int ladder_unperm(int m) {
    constexpr int M = (1 << NQ) - 1;
    return ((m ^ (m << 1)) & M) | (m & ~M);
}

// Layout swap that also leaves the ladder frame: the amplitudes are written
// in stored order and each (lane, r) of the other layout reads its true
// index m from slot pi^-1(m).  The lane and register parts of pi^-1 overlap
// in one bit (RB for LO, 5 for HI), so every read is one of two per-lane
// bases plus a compile-time offset.
template <typename T, int NQ, bool FROM_HI>
__device__ __forceinline__ void relayout_ladder(T* re, T* im, cplx<T>* S, int lane) {
    using From = Lay<NQ, FROM_HI>;
    using To = Lay<NQ, !FROM_HI>;
    constexpr int R = From::R;
    constexpr int SPLIT = FROM_HI ? To::RB : 5;
    const SlotMap<NQ, FROM_HI, kSplitSlots<T>> from(lane);
#pragma unroll
    for (int r = 0; r < R; ++r) S[from(r)] = {re[r], im[r]};
    __syncthreads();
    const int ub = ladder_unperm<NQ>(To::glane(lane));
    const int base0 = pad_slot(ub), base1 = pad_slot(ub ^ (1 << SPLIT));
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int u = ladder_unperm<NQ>(To::greg(r));
        const int off = u & ~(1 << SPLIT);
        const cplx<T> v = S[((u >> SPLIT) & 1 ? base1 : base0) + off + (off >> 5)];
        re[r] = v.re;
        im[r] = v.im;
    }
    __syncthreads();
}

// The same swap on a planar image, one component.
template <typename T, int NQ, bool FROM_HI>
__device__ __forceinline__ void relayout_ladder_plane(T* x, T* P, int lane) {
    using From = Lay<NQ, FROM_HI>;
    using To = Lay<NQ, !FROM_HI>;
    constexpr int R = From::R;
    constexpr int SPLIT = FROM_HI ? To::RB : 5;
    const SlotMap<NQ, FROM_HI, kSplitSlots<T>> from(lane);
#pragma unroll
    for (int r = 0; r < R; ++r) P[from(r)] = x[r];
    __syncthreads();
    const int ub = ladder_unperm<NQ>(To::glane(lane));
    const int base0 = pad_slot(ub), base1 = pad_slot(ub ^ (1 << SPLIT));
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int u = ladder_unperm<NQ>(To::greg(r));
        const int off = u & ~(1 << SPLIT);
        x[r] = P[((u >> SPLIT) & 1 ? base1 : base0) + off + (off >> 5)];
    }
    __syncthreads();
}

template <typename T, int NQ, bool FROM_HI>
__device__ __forceinline__ void relayout_ladder(T* re, T* im, T* P, int lane) {
    relayout_ladder_plane<T, NQ, FROM_HI>(re, P, lane);
    relayout_ladder_plane<T, NQ, FROM_HI>(im, P, lane);
}

// Write the registers (ladder frame) to LDS in natural order: slot pi(k).
// In LO, pi of the register part is prefix(r) in bits 0..RB-1 and the
// parity of r in every higher bit, so again two bases and an offset; HI
// first swaps to LO through relayout_ladder.
template <typename T, int NQ, bool HI>
__device__ __forceinline__ void store_state_ladder(T* re, T* im, cplx<T>* S, int lane) {
    using Lo = Lay<NQ, false>;
    constexpr int R = Lo::R, RB = Lo::RB;
    constexpr int HM = ((1 << NQ) - 1) & ~((1 << RB) - 1);
    if constexpr (HI) relayout_ladder<T, NQ, true>(re, im, S, lane);
    if constexpr (HI) {
        const SlotMap<NQ, false, kSplitSlots<T>> lo(lane);
#pragma unroll
        for (int r = 0; r < R; ++r) S[lo(r)] = {re[r], im[r]};
    } else {
        const int pl = ladder_perm<NQ>(Lo::glane(lane));
        const int base0 = pad_slot(pl), base1 = pad_slot(pl ^ HM);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int off = ladder_perm<NQ>(r) & ((1 << RB) - 1);
            S[(odd_bits(r) ? base1 : base0) + off + (off >> 5)] = {re[r], im[r]};
        }
    }
    __syncthreads();
}

// One component of the registers to a planar image in natural order:
// layout LO, ladder frame (slot pi(k)), or true frame (after a ladder swap
// from HI).
template <typename T, int NQ, bool FRAME>
__device__ __forceinline__ void store_plane_ladder_lo(const T* x, T* P, int lane) {
    using Lo = Lay<NQ, false>;
    constexpr int R = Lo::R, RB = Lo::RB;
    constexpr int HM = ((1 << NQ) - 1) & ~((1 << RB) - 1);
    if constexpr (!FRAME) {
        const SlotMap<NQ, false, kSplitSlots<T>> lo(lane);
#pragma unroll
        for (int r = 0; r < R; ++r) P[lo(r)] = x[r];
    } else {
        const int pl = ladder_perm<NQ>(Lo::glane(lane));
        const int base0 = pad_slot(pl), base1 = pad_slot(pl ^ HM);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int off = ladder_perm<NQ>(r) & ((1 << RB) - 1);
            P[(odd_bits(r) ? base1 : base0) + off + (off >> 5)] = x[r];
        }
    }
    __syncthreads();
}

// Forward pass of the RY + CNOT-ladder ansatz, starting in LO (true frame).
// Layer 0 runs as in the CZ form; a layer that starts in HI (odd) turns
// qubits 5..NQ-1 in the ladder frame, swaps to LO (true frame) and turns
// qubits 0..4; a later layer that starts in LO turns qubits 0..RB-2 in the
// ladder frame, qubit RB-1 too when it is 4 (lane swap), swaps to HI and
// turns the rest.  Ends in the ladder frame, in LO (layers even) or HI.
template <typename T, int NQ, typename Buf>
__device__ __forceinline__ void forward_layers_ladder(T* re, T* im, Buf S, const T* trig, int layers, int lane) {
    constexpr int RB = Lay<NQ, false>::RB;
    ry_range<T, NQ, false, 0, 0, NQ>(re, im, lane, trig, 0);
    relayout<T, NQ, false>(re, im, S, lane);
    ry_range<T, NQ, true, 0, RB, NQ>(re, im, lane, trig, 0);
    int l = 1;
    for (; l < layers; l += 2) {
        // odd layer l: starts in HI
        int kb = l * NQ;
        ry_range_ladder<T, NQ, true, 5, NQ>(re, im, lane, trig, kb);
        relayout_ladder<T, NQ, true>(re, im, S, lane);
        ry_range<T, NQ, false, 0, 0, 5>(re, im, lane, trig, kb);
        if (l + 1 >= layers) break;
        // even layer l + 1: starts in LO
        kb += NQ;
        ry_range_ladder<T, NQ, false, 0, RB - 1>(re, im, lane, trig, kb);
        if constexpr (RB - 1 < 5)
            ry_lane_ladder_lo<T, NQ>(re, im, trig[2 * (kb + RB - 1)], trig[2 * (kb + RB - 1) + 1]);
        relayout_ladder<T, NQ, false>(re, im, S, lane);
        ry_range<T, NQ, true, 0, 5, NQ>(re, im, lane, trig, kb);
    }
}

template <int NQ>
__device__ __forceinline__ bool ladder_flip(int g) {
    constexpr int ladder = (1 << (NQ - 1)) - 1;
    return __popc((unsigned)(g & (g >> 1) & ladder)) & 1;
}

// The CZ-ladder sign (-1)^{Q(g)} of amplitude (lane, r) of a layout.  With
// g = glane | greg(r) on disjoint bits, Q(g) = Q(glane) + Q(greg) + the one
// adjacent pair split between them (lane bit 4 and register bit 0 in HI,
// register bit RB-1 and lane bit 0 in LO): two per-lane bits and
// compile-time register parts, instead of a popcount per amplitude.
template <int NQ, bool HI>
struct LadderSign {
    bool qa, la;
    __device__ __forceinline__ explicit LadderSign(int lane) {
        qa = ladder_flip<NQ>(Lay<NQ, HI>::glane(lane) & ((1 << NQ) - 1));
        la = HI ? ((lane >> 4) & 1) : (lane & 1);
    }
    static constexpr bool qb(int r) {
        return odd_bits(Lay<NQ, HI>::greg(r) & (Lay<NQ, HI>::greg(r) >> 1) & ((1 << (NQ - 1)) - 1));
    }
    static constexpr bool rb(int r) { return HI ? (r & 1) : ((r >> (Lay<NQ, HI>::RB - 1)) & 1); }
    __device__ __forceinline__ bool flip(int r) const { return qa ^ qb(r) ^ (la && rb(r)); }
};

// Write the registers to LDS in natural order, applying S^p (the pending
// CZ-ladder sign) on the way.
template <typename T, int NQ, bool HI>
__device__ __forceinline__ void store_state(const T* re, const T* im, cplx<T>* S, int lane, int p) {
    constexpr int R = Lay<NQ, HI>::R;
    const LadderSign<NQ, HI> ls(lane);
    const SlotMap<NQ, HI, kSplitSlots<T>> sm(lane);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const bool flip = p && ls.flip(r);
        S[sm(r)] = flip ? cplx<T>{-re[r], -im[r]} : cplx<T>{re[r], im[r]};
    }
    __syncthreads();
}

// One component of the registers to a planar image, natural order, S^p applied.
template <typename T, int NQ, bool HI>
__device__ __forceinline__ void store_plane(const T* x, T* P, int lane, int p) {
    constexpr int R = Lay<NQ, HI>::R;
    const LadderSign<NQ, HI> ls(lane);
    const SlotMap<NQ, HI, kSplitSlots<T>> sm(lane);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const bool flip = p && ls.flip(r);
        P[sm(r)] = flip ? -x[r] : x[r];
    }
    __syncthreads();
}

// Forward pass of the ansatz on the registers (both halves), starting in
// layout LO with p = 0.  Ends in LO (layers even) or HI (odd) with
// p = layers mod 2.
template <typename T, int NQ, typename Buf>
__device__ __forceinline__ void forward_layers(T* re, T* im, Buf S, const T* trig, int layers, int lane) {
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

// Rotation parameters of every gate: phi = theta/2 reduced to [-pi/2, pi/2]
// (in float64), then tan(phi/2) and sin(phi) = 2 t / (1 + t^2) in the state
// precision.
template <typename T>
__device__ __forceinline__ void rotation_table(const double* __restrict__ theta, int P, T* trig, int lane) {
    for (int k = lane; k < P; k += 64) {
        double ph = 0.5 * theta[k];
        ph -= 3.14159265358979323846 * rint(ph * 0.31830988618379067154);
        T t;
        if constexpr (sizeof(T) == sizeof(float))
            t = tanf(0.5f * (float)ph);
        else
            t = tan(0.5 * ph);
        trig[2 * k] = t;
        trig[2 * k + 1] = (T)2 * t / fmat(t, t, (T)1);
    }
    __syncthreads();
}

}  // namespace dvq

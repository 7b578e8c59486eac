// Register-resident Hadamard-test kernels: one wavefront simulates one
// (n+1)-qubit circuit of the local cost (Section II-A, II-C, Eq. (4)), with
// the 2^(n+1) amplitudes spread over 64 lanes x 2^(n-5) registers.
//
// Circuit (b = |+>^n, so U_b Z_j U_b^dagger = H^n Z_j H^n = X_j):
//   beta_lm:    H(anc); V(theta); C-A_m; C-A_l; [S^dagger(anc)]; H(anc); <Z_anc>
//   delta^j_lm: H(anc); V(theta); C-A_m; C-X_j; C-A_l; [S^dagger]; H(anc); <Z_anc>
//
// Layout.  Lane bit 5 is the ancilla.  Two layouts alternate:
//   LO: register bits = qubits 0..n-6, lane bits 0..4 = qubits n-5..n-1;
//   HI: register bits = qubits 5..n-1, lane bits 0..4 = qubits 0..4.
// Every layer applies RY to the register qubits of its first layout, swaps
// layouts once through LDS, and applies RY to the remaining qubits, so each
// layer costs one LDS round trip; the next layer starts in the layout the
// previous one ended in.
//
// RY(t) rotates each amplitude pair by phi = t/2.  phi is reduced to
// [-pi/2, pi/2] (a rotation by pi is a global -1, which does not change
// <Z_anc> because V acts on both ancilla halves) and applied as three shears
// a -= tan(phi/2) b; b += sin(phi) a; a -= tan(phi/2) b: six FMAs per
// complex pair.
//
// CZ ladder.  The ladder is the diagonal S = diag((-1)^{Q(g)}),
// Q(g) = sum_q g_q g_{q+1}.  Instead of flipping signs, the kernel keeps the
// stored state psi with true state S^p psi (p = layers applied so far mod 2).
// Conjugating RY_q by S negates its angle on the pairs whose neighbour bits
// g_{q-1} xor g_{q+1} are 1, so an RY in an odd layer uses +-angle per pair;
// the sign is a per-lane value times a compile-time per-register value.  S is
// applied to the amplitudes once, when the state leaves the registers.
//
// Suffix.  The state is written to LDS in natural order (with one pad
// amplitude per 32 to spread banks); the controlled Pauli strings (and X_j)
// act on the ancilla = 1 half as one permutation with phase:
//   (U psi)[k] = omega (-1)^{Z.k} psi[k ^ X]
// (the product of the strings, exact: the phases are powers of i), and each
// lane forms, for its k, a0 = psi0[k], a1 = (U psi1)[k], applies S^dagger,
// the final H and accumulates |a0'|^2 - |a1'|^2.
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
    // global basis index of (lane, r)
    __device__ static __forceinline__ int g(int lane, int r) {
        return HI ? ((lane & 31) | (r << 5) | ((lane >> 5) << NQ))
                  : (r | ((lane & 31) << RB) | ((lane >> 5) << NQ));
    }
};

// LDS slot of basis index g: one pad amplitude every 32.
__device__ __forceinline__ int pad_slot(int g) { return g + (g >> 5); }

template <typename T, int NQ, bool HI, int Q, int PAR>
__device__ __forceinline__ void ry_reg(T* re, T* im, int lane, T t, T s) {
    using Ly = Lay<NQ, HI>;
    constexpr int R = Ly::R;
    constexpr int j = Ly::reg(Q);
    static_assert(j >= 0, "qubit not in registers");
    constexpr int lm = Q > 0 ? Ly::lanebit(Q - 1) : -1;
    constexpr int lp = Q + 1 < NQ ? Ly::lanebit(Q + 1) : -1;
    constexpr int rm = Q > 0 ? Ly::reg(Q - 1) : -1;
    constexpr int rp = Q + 1 < NQ ? Ly::reg(Q + 1) : -1;
    T tp = t, sp = s;
    if constexpr (PAR) {
        int rl = 0;
        if constexpr (lm >= 0) rl ^= lane >> lm;
        if constexpr (lp >= 0) rl ^= lane >> lp;
        if (rl & 1) {
            tp = -t;
            sp = -s;
        }
    }
    const T mtp = -tp, mtn = tp, spp = sp, spn = -sp;
#pragma unroll
    for (int r0 = 0; r0 < R; ++r0) {
        if (r0 & (1 << j)) continue;
        const int r1 = r0 | (1 << j);
        bool neg = false;
        if constexpr (PAR) {
            if (rm >= 0) neg ^= (r0 >> rm) & 1;
            if (rp >= 0) neg ^= (r0 >> rp) & 1;
        }
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

// RY on every qubit q in [Q, QEND) that is a register qubit of the layout.
template <typename T, int NQ, bool HI, int PAR, int Q, int QEND>
__device__ __forceinline__ void ry_range(T* re, T* im, int lane, const T* trig, int kbase) {
    if constexpr (Q < QEND) {
        if constexpr (Lay<NQ, HI>::reg(Q) >= 0) {
            const T t = trig[2 * (kbase + Q)], s = trig[2 * (kbase + Q) + 1];
            ry_reg<T, NQ, HI, Q, PAR>(re, im, lane, t, s);
        }
        ry_range<T, NQ, HI, PAR, Q + 1, QEND>(re, im, lane, trig, kbase);
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

// Write the registers to LDS in natural order, applying S^p (the pending
// CZ-ladder sign) on the way.
template <typename T, int NQ, bool HI>
__device__ __forceinline__ void store_state(const T* re, const T* im, cplx<T>* S, int lane, int p) {
    constexpr int R = Lay<NQ, HI>::R;
    constexpr int ladder = (1 << (NQ - 1)) - 1;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int g = Lay<NQ, HI>::g(lane, r);
        const bool flip = p && (__popc((unsigned)(g & (g >> 1) & ladder)) & 1);
        S[pad_slot(g)] = flip ? cplx<T>{-re[r], -im[r]} : cplx<T>{re[r], im[r]};
    }
    __syncthreads();
}

template <typename T, int NQ>
__global__ void __launch_bounds__(64) k_terms_fast(TermsArgs g) {
    constexpr int R = Lay<NQ, false>::R;
    constexpr int N = 1 << NQ;
    constexpr int NSLOT = 2 * N + (2 * N) / 32;
    extern __shared__ __align__(16) unsigned char smem[];
    cplx<T>* S = reinterpret_cast<cplx<T>*>(smem);
    T* trig = reinterpret_cast<T*>(S + NSLOT);
    const int lane = threadIdx.x;
    const int layers = g.layers, P = NQ * layers;

    const int64_t gid = (int64_t)blockIdx.x + (int64_t)blockIdx.y * gridDim.x;
    if (gid >= g.total) return;
    const int64_t row = gid / g.per_row;
    const Term t = decode_term(gid - row * g.per_row, g.L, NQ, g.kind);

    // Rotation parameters of every gate: phi = theta/2 reduced to [-pi/2, pi/2].
    for (int k = lane; k < P; k += 64) {
        double ph = 0.5 * g.theta[row * P + k];
        ph -= 3.14159265358979323846 * rint(ph * 0.31830988618379067154);
        trig[2 * k] = (T)tan(0.5 * ph);
        trig[2 * k + 1] = (T)sin(ph);
    }
    __syncthreads();

    // |0> with H on the ancilla: 1/sqrt(2) at g = 0 and g = 2^n (layout LO).
    T re[R], im[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        re[r] = (r == 0 && (lane & 31) == 0) ? (T)0.70710678118654752440 : (T)0;
        im[r] = (T)0;
    }

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
        store_state<T, NQ, true>(re, im, S, lane, 1);  // odd number of ladders
    } else {
        store_state<T, NQ, false>(re, im, S, lane, 0);
    }

    // Controlled U = A_l [X_j] A_m on the ancilla = 1 half as one signed permutation.
    const dvq_pauli pl = g.strings[t.l], pm = g.strings[t.m];
    const uint32_t xmid = pl.x ^ (t.type == kDelta ? (1u << t.j) : 0u);
    const uint32_t X = xmid ^ pm.x, Z = pl.z ^ pm.z;
    const int pw = (int)__popc(pl.x & pl.z) + (int)__popc(pm.x & pm.z) +
                   2 * (int)((__popc(pl.z & pl.x) + __popc(pm.z & X)) & 1);
    const T r2 = (T)0.70710678118654752440;
    T z = 0;
#pragma unroll 4
    for (int i = 0; i < N / 64; ++i) {
        const int k = lane + 64 * i;
        const cplx<T> a0 = S[pad_slot(k)];
        cplx<T> a1 = mul_ipow(S[pad_slot(N + (k ^ (int)X))],
                              pw + 2 * (int)(__popc((unsigned)k & Z) & 1) + (t.part ? 3 : 0));
        const T b0r = (a0.re + a1.re) * r2, b0i = (a0.im + a1.im) * r2;
        const T b1r = (a0.re - a1.re) * r2, b1i = (a0.im - a1.im) * r2;
        z += (b0r * b0r + b0i * b0i) - (b1r * b1r + b1i * b1i);
    }
    z = wave_sum(z);
    if (lane == 0) store_term(g, row, t, (double)z);
}

template <typename T, int NQ>
static dvq_status launch_fast(const TermsArgs& g, hipStream_t s) {
    constexpr int N = 1 << NQ;
    const size_t lds = (size_t)(2 * N + (2 * N) / 32) * sizeof(cplx<T>) +
                       (size_t)2 * NQ * g.layers * sizeof(T);
    DVQ_TRY_HIP(allow_lds((const void*)k_terms_fast<T, NQ>, lds));
    hipLaunchKernelGGL((k_terms_fast<T, NQ>), grid_for(g.total), dim3(64), lds, s, g);
    DVQ_CHECK_LAUNCH("k_terms_fast");
    return DVQ_OK;
}

dvq_status launch_terms_fast(const TermsArgs& g, int precision, hipStream_t s) {
    if (g.kind != DVQ_COST_LOCAL || g.bkind != DVQ_B_PLUS || g.ent != DVQ_ENT_CZ_LADDER)
        return DVQ_EUNSUPPORTED;
    if (g.n * g.layers > 1024) return DVQ_EUNSUPPORTED;
    if (precision == DVQ_F32) {
        if (g.n == 10) return launch_fast<float, 10>(g, s);
        if (g.n == 11) return launch_fast<float, 11>(g, s);
    } else {
        if (g.n == 10) return launch_fast<double, 10>(g, s);
    }
    return DVQ_EUNSUPPORTED;
}

}  // namespace dvq

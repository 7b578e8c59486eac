// Register-resident Hadamard-test kernels: one wavefront simulates one
// (n+1)-qubit circuit of the local cost (Section II-A, II-C, Eq. (4)), with
// the 2^(n+1) amplitudes spread over 64 lanes x 2^(n-5) registers.
//
// Circuit (b = |+>^n, so U_b Z_j U_b^dagger = H^n Z_j H^n = X_j):
//   beta_lm:    H(anc); V(theta); C-A_m; C-A_l; [S^dagger(anc)]; H(anc); <Z_anc>
//   delta^j_lm: H(anc); V(theta); C-A_m; C-X_j; C-A_l; [S^dagger]; H(anc); <Z_anc>
// For a general real b, C-X_j becomes C-(U_b Z_j U_b^dagger) with the
// Householder U_b (measure_suffix_bvec).
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
// CNOT ladder.  The same kernels run the RY + CNOT-ladder ansatz: the ladder
// is a permutation, carried as a frame on the registers and applied when
// the state next goes through LDS (forward_layers_ladder).
//
// Suffix.  The state is written to LDS in natural order (with one pad
// amplitude per 32 to spread banks); the controlled Pauli strings (and X_j)
// act on the ancilla = 1 half as one permutation with phase:
//   (U psi)[k] = omega (-1)^{Z.k} psi[k ^ X]
// (the product of the strings, exact: the phases are powers of i), and each
// lane forms, for its k, a0 = psi0[k], a1 = (U psi1)[k]; S^dagger, the final
// H and <Z_anc> give |a0 + a1'|^2 - |a0 - a1'|^2 (unnormalised), which the
// kernels evaluate as 4 Re(conj(a0) a1') (z_sums, measure_planar).
#include "circuits.h"
#include "wave_state.h"

namespace dvq {

// The shared prefix of every circuit of one theta row: H on the ancilla and
// V(theta) on the system register, left in LDS (natural order, padded) with
// the pending ladder (sign or permutation) applied.  `trig` receives the
// rotation parameters phi = theta/2 reduced to [-pi/2, pi/2]: tan(phi/2),
// sin(phi).
// The prefix in registers: |0> with H on the ancilla (1/sqrt(2) at g = 0
// and g = 2^n, layout LO), then V(theta), swapping layouts through the LDS
// image S (interleaved cplx<T>* or planar T*).  Ends as forward_layers /
// forward_layers_ladder leave it.  The layout swaps address S with
// `slot_lane`: the lane itself, or lane & 31 to fold the two ancilla halves
// (identical until the controlled gates) onto one image.
template <typename T, int NQ, int ENT, typename Buf>
__device__ __forceinline__ void prefix_from_table(int layers, Buf S, const T* trig, int lane, int slot_lane, T* re,
                                                  T* im) {
    constexpr int R = Lay<NQ, false>::R;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        re[r] = (r == 0 && (lane & 31) == 0) ? (T)0.70710678118654752440 : (T)0;
        im[r] = (T)0;
    }
    if constexpr (ENT == DVQ_ENT_CZ_LADDER)
        forward_layers<T, NQ>(re, im, S, trig, layers, slot_lane);
    else
        forward_layers_ladder<T, NQ>(re, im, S, trig, layers, slot_lane);
}

template <typename T, int NQ, int ENT, typename Buf>
__device__ __forceinline__ void prefix_registers(const double* __restrict__ theta, int layers, Buf S, T* trig,
                                                 int lane, int slot_lane, T* re, T* im) {
    rotation_table<T>(theta, NQ * layers, trig, lane);
    prefix_from_table<T, NQ, ENT>(layers, S, trig, lane, slot_lane, re, im);
}

template <typename T, int NQ, int ENT>
__device__ __forceinline__ void simulate_prefix(const double* __restrict__ theta, int layers,
                                                cplx<T>* S, T* trig, int lane) {
    constexpr int R = Lay<NQ, false>::R;
    T re[R], im[R];
    prefix_registers<T, NQ, ENT>(theta, layers, S, trig, lane, lane, re, im);
    if constexpr (ENT == DVQ_ENT_CZ_LADDER) {
        if (layers & 1)
            store_state<T, NQ, true>(re, im, S, lane, 1);
        else
            store_state<T, NQ, false>(re, im, S, lane, 0);
    } else {
        if (layers & 1)
            store_state_ladder<T, NQ, true>(re, im, S, lane);
        else
            store_state_ladder<T, NQ, false>(re, im, S, lane);
    }
}

// Controlled U = A_l [X_j] A_m on the ancilla = 1 half as one signed
// permutation: (U psi)[k] = i^pw (-1)^{Z.k} psi[k ^ X].
struct SignedPerm {
    uint32_t X, Z;
    int pw;
};

__device__ __forceinline__ SignedPerm suffix_perm(const dvq_pauli pl, const dvq_pauli pm, int type, int j) {
    const uint32_t xmid = pl.x ^ (type == kDelta ? (1u << j) : 0u);
    SignedPerm sp;
    sp.X = xmid ^ pm.x;
    sp.Z = pl.z ^ pm.z;
    sp.pw = (int)__popc(pl.x & pl.z) + (int)__popc(pm.x & pm.z) +
            2 * (int)((__popc(pl.z & pl.x) + __popc(pm.z & sp.X)) & 1);
    return sp;
}

// Basis state k = lane + 64 i of the lane's i-th amplitude: k ^ X and the
// parity of k & Z split into a per-lane part and a part uniform over the
// wavefront (i, X >> 6, Z >> 6), so the loop body needs one address add and
// one phase add per amplitude.
struct SuffixLane {
    int base;  // pad_slot offset of (lane ^ (X & 63)) within a half
    int pw;    // phase power from the lane bits
    int xh, zh;
};

__device__ __forceinline__ SuffixLane suffix_lane(const SignedPerm& sp, int lane) {
    SuffixLane sl;
    const int b = lane ^ (int)(sp.X & 63u);
    sl.base = b + (b >> 5);
    sl.pw = sp.pw + 2 * (int)(__popc((unsigned)lane & (sp.Z & 63u)) & 1);
    sl.xh = (int)(sp.X >> 6);
    sl.zh = (int)(sp.Z >> 6);
    return sl;
}

// pad_slot(src + ((lane ^ X) + 64 (i ^ xh))) = pad_slot(src) + base + 66 (i ^ xh)
// (src a multiple of 64, lane ^ (X & 63) < 64).
__device__ __forceinline__ int suffix_slot(const SuffixLane& sl, int src, int i) {
    return src + (src >> 5) + sl.base + 66 * (i ^ sl.xh);
}

__device__ __forceinline__ int suffix_pow(const SuffixLane& sl, int i) {
    return sl.pw + 2 * (int)(__popc((unsigned)(i & sl.zh)) & 1);
}

// The phase i^p of the controlled string at amplitude i of a lane,
// p = pw(lane) + 2 parity(i & zh) (+ 3 for S^dagger): a per-lane rotation
// i^q = c + i d, the same for every i, times a sign uniform over the wave.
template <typename T>
struct PhaseSplit {
    T c, d;
    __device__ __forceinline__ PhaseSplit(const SuffixLane& sl, int imag) {
        const int q = (sl.pw + (imag ? 3 : 0)) & 3;
        c = (T)((q == 0) - (q == 2));
        d = (T)((q == 1) - (q == 3));
    }
};

// One amplitude pair's share of <Z_anc> after the controlled string (phase
// i^q times `sgn`, the permuted amplitude g) and the final H, applied
// unnormalised (the two 1/sqrt(2) factors are applied once to the wave's
// sum): |a0 + a1|^2 - |a0 - a1|^2 = 4 Re(conj(a0) a1) with a1 = sgn i^q g,
// i^q = c + i d.  Summed over the pairs this is 4 (c S1 + d S2) with
// S1 = sum sgn (a0r gr + a0i gi), S2 = sum sgn (a0i gr - a0r gi), which
// serve the real and the imaginary circuit of a term alike.
template <typename T>
__device__ __forceinline__ void z_sums(T a0r, T a0i, T gr, T gi, T sgn, T& s1, T& s2) {
    s1 = fmat(sgn, fmat(a0r, gr, a0i * gi), s1);
    s2 = fmat(sgn, fmat(a0i, gr, -(a0r * gi)), s2);
}

// <Z_anc> after applying U to the ancilla = 1 half, S^dagger (imag) and the
// final H, summed over the lane's basis states and reduced over the wave.
template <typename T, int NQ>
__device__ __forceinline__ T measure_suffix(const cplx<T>* S, SignedPerm sp, int imag, int lane) {
    constexpr int N = 1 << NQ;
    const SuffixLane sl = suffix_lane(sp, lane);
    const PhaseSplit<T> ph(sl, imag);
    T s1 = 0, s2 = 0;
#pragma unroll 4
    for (int i = 0; i < N / 64; ++i) {
        const cplx<T> a0 = S[pad_slot(lane + 64 * i)];
        const cplx<T> g = S[suffix_slot(sl, N, i)];
        const T sgn = (__popc((unsigned)(i & sl.zh)) & 1) ? (T)-1 : (T)1;
        z_sums(a0.re, a0.im, g.re, g.im, sgn, s1, s2);
    }
    return (T)2 * wave_sum(fmat(ph.c, s1, ph.d * s2));
}

// Both circuits (real, imaginary) of one term from one pass over the state:
// the gathers and phases are shared, each circuit gets its own S^dagger,
// H and <Z_anc>.
// `src` is the offset of the half the controlled gates read (N: the
// ancilla = 1 half; 0: the other half, which holds the same amplitudes,
// when half 1 serves as scratch).
template <typename T, int NQ>
__device__ __forceinline__ void measure_suffix_pair(const cplx<T>* S, SignedPerm sp, int lane, T& zre,
                                                    T& zim, int src = 1 << NQ) {
    constexpr int N = 1 << NQ;
    const SuffixLane sl = suffix_lane(sp, lane);
    const PhaseSplit<T> pre(sl, 0), pim(sl, 1);  // real-part circuit; imaginary part (S^dagger)
    T s1 = 0, s2 = 0;
#pragma unroll 4
    for (int i = 0; i < N / 64; ++i) {
        const cplx<T> a0 = S[pad_slot(lane + 64 * i)];
        const cplx<T> g = S[suffix_slot(sl, src, i)];
        const T sgn = (__popc((unsigned)(i & sl.zh)) & 1) ? (T)-1 : (T)1;
        z_sums(a0.re, a0.im, g.re, g.im, sgn, s1, s2);
    }
    zre = (T)2 * wave_sum(fmat(pre.c, s1, pre.d * s2));
    zim = (T)2 * wave_sum(fmat(pim.c, s1, pim.d * s2));
}

// measure_suffix on a planar image, from the registers prefix_registers
// left: the final state goes to LDS one component at a time (with the
// pending ladder sign or frame), both ancilla halves onto one image (they are
// equal before the controlled gates; the lanes of the upper half write the
// same values as those of the lower).  After the real parts each lane keeps
// its ancilla = 0 amplitudes' real parts and the real parts of the permuted
// ancilla = 1 amplitudes; with the imaginary parts it completes each pair
// and applies the same S^dagger / H / <Z_anc> as measure_suffix.  The
// registers are as prefix_registers left them, except that with the CNOT
// ladder at odd depth the caller has swapped them from HI (ladder frame) to
// LO (true frame) first.
template <typename T, int NQ, int ENT>
__device__ __forceinline__ void store_final_plane(const T* x, T* P, int layers, int lane) {
    if constexpr (ENT == DVQ_ENT_CZ_LADDER) {
        if (layers & 1)
            store_plane<T, NQ, true>(x, P, lane, 1);
        else
            store_plane<T, NQ, false>(x, P, lane, 0);
    } else {
        if (layers & 1)
            store_plane_ladder_lo<T, NQ, false>(x, P, lane);
        else
            store_plane_ladder_lo<T, NQ, true>(x, P, lane);
    }
}

template <typename T, int NQ, int ENT>
__device__ __forceinline__ T measure_planar(T* re, T* im, T* P, SignedPerm sp, int imag, int layers, int lane) {
    constexpr int N = 1 << NQ, KPL = N / 64;
    const SuffixLane sl = suffix_lane(sp, lane);
    // pad_slot(lane + 64 i) = a0 + 66 i: one base, the offsets are immediates
    const int a0 = lane + (lane >> 5);
    T a0r[KPL], gr[KPL];
    store_final_plane<T, NQ, ENT>(re, P, layers, lane & 31);
#pragma unroll
    for (int i = 0; i < KPL; ++i) {
        a0r[i] = P[a0 + 66 * i];
        gr[i] = P[suffix_slot(sl, 0, i)];
    }
    __syncthreads();  // every lane has read the real parts
    store_final_plane<T, NQ, ENT>(im, P, layers, lane & 31);
    // The gather addresses are formed again for the imaginary parts (one
    // add each) instead of being held in registers across the store above.
    SuffixLane sl2 = sl;
    asm volatile("" : "+v"(sl2.base));
    // |a0 + a1|^2 - |a0 - a1|^2 = 4 Re(conj(a0) a1), a1 = sgn (c + i d) g:
    // 4 sgn (c (a0r gr + a0i gi) + d (a0i gr - a0r gi)).  One of c, d is zero,
    // the same one in every lane (the lane part of the phase only flips its
    // sign), so each amplitude pair needs one product pair, and the lane's
    // c or d multiplies its sum once.
    const PhaseSplit<T> ph(sl, imag);
    const bool odd = (sp.pw + (imag ? 3 : 0)) & 1;  // wave-uniform: d != 0
    T z = 0;
    if (!odd) {
#pragma unroll
        for (int i = 0; i < KPL; ++i) {
            const T a0i = P[a0 + 66 * i], gi = P[suffix_slot(sl2, 0, i)];
            const T sgn = (__popc((unsigned)(i & sl.zh)) & 1) ? (T)-1 : (T)1;
            z = fmat(sgn, fmat(a0r[i], gr[i], a0i * gi), z);
        }
        z *= ph.c;
    } else {
#pragma unroll
        for (int i = 0; i < KPL; ++i) {
            const T a0i = P[a0 + 66 * i], gi = P[suffix_slot(sl2, 0, i)];
            const T sgn = (__popc((unsigned)(i & sl.zh)) & 1) ? (T)-1 : (T)1;
            z = fmat(sgn, fmat(a0i, gr[i], -(a0r[i] * gi)), z);
        }
        z *= ph.d;
    }
    return (T)2 * wave_sum(z);
}

// Phase power of one Pauli string: (P v)[k] = i^p (-1)^{z.k} v[k ^ x] with
// p = |x&z| + 2 (|x&z| mod 2) (P = i^{|x&z|} X^x Z^z).
__device__ __forceinline__ int string_pow(const dvq_pauli ps) {
    const int c = (int)__popc(ps.x & ps.z);
    return c + 2 * (c & 1);
}

// delta^j_lm for a general real unit b (Householder U_b, U_b = U_b^dagger up
// to a sign that cancels): U = A_l (H Z_j H) A_m with H = I - 2 w w^T / w^T w,
// w = e_0 - s b.  On u = A_m psi,
//   H Z_j H u = Z_j u + w (c1 + sigma c2),  sigma_k = (-1)^{k_j},
//   c1 = -2 beta / om + 4 zeta alpha / om^2,  c2 = -2 alpha / om,
//   alpha = w.u, beta = w.(Z_j u), zeta = w.(Z_j w), om = w.w,
// so the circuit is one gather (u, into registers), five wave sums, one
// write of H Z_j H u into the ancilla = 1 half of LDS and one gather of A_l
// of it; then S^dagger / H / <Z_anc> for both parts as in
// measure_suffix_pair.  `src` as there; the ancilla = 1 half is overwritten.
template <typename T, int NQ>
__device__ __forceinline__ void measure_suffix_bvec(cplx<T>* S, dvq_pauli pl, dvq_pauli pm, int j,
                                                    const double* __restrict__ b, int lane, T& zre, T& zim,
                                                    int src) {
    constexpr int N = 1 << NQ, KPL = N / 64;
    const double sg = (b[0] > 0.0) ? -1.0 : 1.0;
    const int pwm = string_pow(pm);
    cplx<T> u[KPL];
    T ar = 0, ai = 0, br = 0, bi = 0, ze = 0, om = 0;
#pragma unroll
    for (int i = 0; i < KPL; ++i) {
        const int k = lane + 64 * i;
        u[i] = mul_ipow(S[pad_slot(src + (k ^ (int)pm.x))], pwm + 2 * (int)(__popc((unsigned)k & pm.z) & 1));
        const T w = (T)((k == 0 ? 1.0 : 0.0) - sg * b[k]);
        const T sw = ((k >> j) & 1) ? -w : w;
        ar += w * u[i].re;
        ai += w * u[i].im;
        br += sw * u[i].re;
        bi += sw * u[i].im;
        ze += sw * w;
        om += w * w;
    }
    ar = wave_sum(ar);
    ai = wave_sum(ai);
    br = wave_sum(br);
    bi = wave_sum(bi);
    ze = wave_sum(ze);
    om = wave_sum(om);
    const T io = (T)1 / om;
    const T f = (T)4 * ze * io * io;
    const T c1r = -(T)2 * br * io + f * ar, c1i = -(T)2 * bi * io + f * ai;
    const T c2r = -(T)2 * ar * io, c2i = -(T)2 * ai * io;
    __syncthreads();  // every lane has read its u
#pragma unroll
    for (int i = 0; i < KPL; ++i) {
        const int k = lane + 64 * i;
        const T w = (T)((k == 0 ? 1.0 : 0.0) - sg * b[k]);
        const bool neg = (k >> j) & 1;
        const T vr = neg ? -u[i].re : u[i].re, vi = neg ? -u[i].im : u[i].im;
        const T er = neg ? c1r - c2r : c1r + c2r, ei = neg ? c1i - c2i : c1i + c2i;
        S[pad_slot(N + k)] = {vr + w * er, vi + w * ei};
    }
    __syncthreads();
    SignedPerm sp;
    sp.X = pl.x;
    sp.Z = pl.z;
    sp.pw = string_pow(pl);
    measure_suffix_pair<T, NQ>(S, sp, lane, zre, zim, N);
}

// measure_suffix_bvec on a planar image, from the registers prefix_registers
// left (literal kernel, one part per circuit).  The final state goes to LDS
// one component at a time; each lane keeps its ancilla = 0 amplitudes and
// gathers u = A_m psi_1; the wave sums give H Z_j H u in registers, which
// goes back through the ancilla = 1 half of the image one component at a
// time, gathered through A_l and measured as in measure_planar.
template <typename T, int NQ, int ENT>
__device__ __forceinline__ T measure_planar_bvec(T* re, T* im, T* P, dvq_pauli pl, dvq_pauli pm, int j,
                                                 const double* __restrict__ b, int imag, int layers, int lane) {
    constexpr int N = 1 << NQ, KPL = N / 64;
    const double sg = (b[0] > 0.0) ? -1.0 : 1.0;
    const int pwm = string_pow(pm);
    // pad_slot(lane + 64 i) = a0 + 66 i and pad_slot(N + (k ^ X_m)) =
    // pad_slot(N) + um + 66 (i ^ (X_m >> 6)): per-lane bases, immediate or
    // wave-uniform offsets; the gather addresses are formed again after each
    // barrier rather than held in registers across the plane stores.
    const int a0 = lane + (lane >> 5);
    const int bm = lane ^ (int)(pm.x & 63u), xhm = (int)(pm.x >> 6);
    int um = bm + (bm >> 5);
    T a0r[KPL], a0i[KPL], ur[KPL], ui[KPL];
    store_final_plane<T, NQ, ENT>(re, P, layers, lane & 31);
#pragma unroll
    for (int i = 0; i < KPL; ++i) {
        a0r[i] = P[a0 + 66 * i];
        ur[i] = P[um + 66 * (i ^ xhm)];
    }
    __syncthreads();  // every lane has read the real parts
    store_final_plane<T, NQ, ENT>(im, P, layers, lane & 31);
    asm volatile("" : "+v"(um));
#pragma unroll
    for (int i = 0; i < KPL; ++i) {
        a0i[i] = P[a0 + 66 * i];
        ui[i] = P[um + 66 * (i ^ xhm)];
    }
    __syncthreads();  // every lane has read the imaginary parts
    T ar = 0, ai = 0, br = 0, bi = 0, ze = 0, om = 0;
#pragma unroll
    for (int i = 0; i < KPL; ++i) {
        const int k = lane + 64 * i;
        const cplx<T> u = mul_ipow(cplx<T>{ur[i], ui[i]}, pwm + 2 * (int)(__popc((unsigned)k & pm.z) & 1));
        ur[i] = u.re;
        ui[i] = u.im;
        const T w = (T)((k == 0 ? 1.0 : 0.0) - sg * b[k]);
        const T sw = ((k >> j) & 1) ? -w : w;
        ar += w * u.re;
        ai += w * u.im;
        br += sw * u.re;
        bi += sw * u.im;
        ze += sw * w;
        om += w * w;
    }
    ar = wave_sum(ar);
    ai = wave_sum(ai);
    br = wave_sum(br);
    bi = wave_sum(bi);
    ze = wave_sum(ze);
    om = wave_sum(om);
    const T io = (T)1 / om;
    const T f = (T)4 * ze * io * io;
    const T c1r = -(T)2 * br * io + f * ar, c1i = -(T)2 * bi * io + f * ai;
    const T c2r = -(T)2 * ar * io, c2i = -(T)2 * ai * io;
    // v = H Z_j H u, in place of u
#pragma unroll
    for (int i = 0; i < KPL; ++i) {
        const int k = lane + 64 * i;
        const T w = (T)((k == 0 ? 1.0 : 0.0) - sg * b[k]);
        const bool neg = (k >> j) & 1;
        const T er = neg ? c1r - c2r : c1r + c2r, ei = neg ? c1i - c2i : c1i + c2i;
        ur[i] = (neg ? -ur[i] : ur[i]) + w * er;
        ui[i] = (neg ? -ui[i] : ui[i]) + w * ei;
    }
    SignedPerm sp;
    sp.X = pl.x;
    sp.Z = pl.z;
    sp.pw = string_pow(pl);
    const SuffixLane sl = suffix_lane(sp, lane);
    T gr[KPL];
#pragma unroll
    for (int i = 0; i < KPL; ++i) P[a0 + 66 * i] = ur[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < KPL; ++i) gr[i] = P[suffix_slot(sl, 0, i)];
    __syncthreads();  // every lane has read the real parts of A_l v
#pragma unroll
    for (int i = 0; i < KPL; ++i) P[a0 + 66 * i] = ui[i];
    __syncthreads();
    SuffixLane sl2 = sl;
    asm volatile("" : "+v"(sl2.base));
    const PhaseSplit<T> ph(sl, imag);
    T s1 = 0, s2 = 0;
#pragma unroll
    for (int i = 0; i < KPL; ++i) {
        const T sgn = (__popc((unsigned)(i & sl.zh)) & 1) ? (T)-1 : (T)1;
        z_sums(a0r[i], a0i[i], gr[i], P[suffix_slot(sl2, 0, i)], sgn, s1, s2);
    }
    return (T)2 * wave_sum(fmat(ph.c, s1, ph.d * s2));
}

// Literal form: one wavefront simulates one circuit, every gate (both
// ancilla halves in registers).  Until the controlled gates the two halves
// hold the same amplitudes, so the layout swaps and the final measurement go
// through one planar image of a single half (N + N/32 values, 4.2 KB in
// float32 at n = 10): the register count alone sets the occupancy.  Float32,
// n <= 10: five wavefronts per SIMD for b = |+> (96 VGPRs), four for a
// general b (126 VGPRs), both ladders, no spill; larger states and float64
// take no bound (a bound would spill heavily).
template <typename T, int NQ, int ENT, bool BVEC>
constexpr int fast_waves() {
    if (sizeof(T) != 4 || NQ > 10) return 1;
    return BVEC ? 4 : 5;
}

// Circuits per wavefront of the literal kernel: in float64 (b = |+>) the two
// circuits of one term share the rotation parameters, 2 % faster per
// evaluation.  The float32 kernels keep one: with two, the CNOT ladder spills,
// the CZ ladder gained 0.5 % while its result writes left the L2s as 4.6 times
// the result bytes, and the general-b kernels would not fit their registers.
template <typename T, int ENT, bool BVEC>
constexpr int circuits_per_wave() {
    return (BVEC || sizeof(T) == 4) ? 1 : 2;
}

// Workgroup b of a launch runs on XCD b mod 8: the dispatcher deals
// workgroups to the eight XCDs in turn, and each XCD has its own L2.  Mapping
// each XCD's workgroups to one contiguous range of circuits keeps neighbouring
// 8-byte results (the two parts of a term, then the next term) in one L2, so
// they leave it as whole 32-byte sectors instead of one partial sector each.
// A bijection of [0, G) for any G.
__device__ __forceinline__ int64_t xcd_contiguous(int64_t b, int64_t G) {
    constexpr int64_t kXcds = 8;
    const int64_t q = G / kXcds, r = G % kXcds, x = b % kXcds;
    return x * q + (x < r ? x : r) + b / kXcds;
}

template <typename T, int NQ, int ENT, bool BVEC>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(fast_waves<T, NQ, ENT, BVEC>()))) k_terms_fast(TermsArgs g) {
    constexpr int N = 1 << NQ;
    constexpr int NSLOT = N + N / 32;  // one ancilla half (the halves are folded)
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x;
    const int P = NQ * g.layers;

    // With two circuits per wavefront, one wavefront per term: its
    // real-part and imaginary-part circuits, each simulated from |0> gate by
    // gate; only the rotation parameters (a function of theta alone) are
    // computed once for both.
    constexpr int CPW = circuits_per_wave<T, ENT, BVEC>();
    const int64_t pid = xcd_contiguous((int64_t)blockIdx.x + (int64_t)blockIdx.y * gridDim.x,
                                       (int64_t)gridDim.x * gridDim.y);
    const int64_t gid = CPW * pid;  // c0 and per_row are even: a pair lies in one row and one term
    if (gid >= g.total) return;
    int64_t row;
    Term t;
    if (g.fast_div) {
        const uint32_t r = div_fast((uint32_t)gid, g.div_row);
        row = r;
        t = decode_term_fast((uint32_t)g.c0 + (uint32_t)gid - r * (uint32_t)g.per_row, g);
    } else {
        row = gid / g.per_row;
        t = decode_term(g.c0 + gid - row * g.per_row, g.L, NQ, g.kind);
    }

    T* Pl = reinterpret_cast<T*>(smem);
    T* trig = Pl + NSLOT;
    constexpr int R = Lay<NQ, false>::R;
    if constexpr (CPW == 1) {
        T re[R], im[R];
        prefix_registers<T, NQ, ENT>(g.theta + row * P, g.layers, Pl, trig, lane, lane & 31, re, im);
        // the measurements start in layout LO (true frame for the CNOT
        // ladder); once here rather than in each, so both share one register
        // assignment
        if constexpr (ENT != DVQ_ENT_CZ_LADDER)
            if (g.layers & 1) relayout_ladder<T, NQ, true>(re, im, Pl, lane & 31);  // HI ladder frame -> LO true frame
        T z;
        if (BVEC && t.type == kDelta) {
            z = measure_planar_bvec<T, NQ, ENT>(re, im, Pl, g.strings[t.l], g.strings[t.m], t.j, g.b, t.part,
                                                g.layers, lane);
        } else {
            const SignedPerm sp = suffix_perm(g.strings[t.l], g.strings[t.m], t.type, t.j);
            z = measure_planar<T, NQ, ENT>(re, im, Pl, sp, t.part, g.layers, lane);
        }
        if (lane == 0) store_term(g, row, t, (double)z);
    } else {
        rotation_table<T>(g.theta + row * P, P, trig, lane);  // ends with a barrier
        T zp[2];
#pragma unroll 1
        for (int part = 0; part < 2; ++part) {
            T re[R], im[R];
            prefix_from_table<T, NQ, ENT>(g.layers, Pl, trig, lane, lane & 31, re, im);
            if constexpr (ENT != DVQ_ENT_CZ_LADDER)
                if (g.layers & 1) relayout_ladder<T, NQ, true>(re, im, Pl, lane & 31);
            const SignedPerm sp = suffix_perm(g.strings[t.l], g.strings[t.m], t.type, t.j);
            zp[part] = measure_planar<T, NQ, ENT>(re, im, Pl, sp, part, g.layers, lane);
            __syncthreads();  // the image is rewritten by the next circuit's first layout swap
        }
        if (lane == 0) store_term_pair(g, row, t, (double)zp[0], (double)zp[1]);
    }
}

// Prefix-shared form: one wavefront simulates the common prefix (H, V(theta))
// once and then the distinct suffix of `chunk` consecutive circuits of the
// same row (whole Re/Im pairs).  Same results as the literal form; the
// ansatz work is paid once per chunk instead of once per circuit.
template <typename T, int NQ, int ENT, bool BVEC>
__global__ void __launch_bounds__(64) k_terms_shared(TermsArgs g, int64_t chunk, int64_t chunks_per_row) {
    constexpr int N = 1 << NQ;
    constexpr int NSLOT = 2 * N + (2 * N) / 32;
    extern __shared__ __align__(16) unsigned char smem[];
    cplx<T>* S = reinterpret_cast<cplx<T>*>(smem);
    T* trig = reinterpret_cast<T*>(S + NSLOT);
    const int lane = threadIdx.x;
    const int P = NQ * g.layers;

    const int64_t wg = (int64_t)blockIdx.x + (int64_t)blockIdx.y * gridDim.x;
    const int64_t row = wg / chunks_per_row;
    if (row >= g.B) return;
    const int64_t c0 = (wg - row * chunks_per_row) * chunk;
    const int64_t c1 = c0 + chunk < g.per_row ? c0 + chunk : g.per_row;

    simulate_prefix<T, NQ, ENT>(g.theta + row * P, g.layers, S, trig, lane);
    for (int64_t c = c0; c < c1; c += 2) {
        const Term t = decode_term(g.c0 + c, g.L, NQ, g.kind);
        T zr, zi;
        if (BVEC && t.type == kDelta) {
            // reads half 0, uses half 1 as scratch
            measure_suffix_bvec<T, NQ>(S, g.strings[t.l], g.strings[t.m], t.j, g.b, lane, zr, zi, 0);
        } else {
            const SignedPerm sp = suffix_perm(g.strings[t.l], g.strings[t.m], t.type, t.j);
            measure_suffix_pair<T, NQ>(S, sp, lane, zr, zi, BVEC ? 0 : N);
        }
        if (lane == 0) {
            store_term(g, row, t, (double)zr);
            Term ti = t;
            ti.part = 1;
            store_term(g, row, ti, (double)zi);
        }
    }
}

// LDS of the literal kernel (planar, folded: N (+ pad) values and the
// rotation table) or of the prefix-shared kernel (interleaved, both halves).
template <typename T, int NQ>
static size_t fast_lds_bytes(int layers, bool folded_planar = false) {
    constexpr int N = 1 << NQ;
    return (folded_planar ? (size_t)(N + N / 32) * sizeof(T) : (size_t)(2 * N + (2 * N) / 32) * sizeof(cplx<T>)) +
           (size_t)2 * NQ * layers * sizeof(T);
}

template <typename T, int NQ, int ENT, bool BVEC>
static dvq_status launch_fast_ent(const TermsArgs& g, hipStream_t s) {
    const size_t lds = fast_lds_bytes<T, NQ>(g.layers, true);
    DVQ_TRY_HIP(allow_lds((const void*)k_terms_fast<T, NQ, ENT, BVEC>, lds));
    if ((g.c0 | g.per_row) & 1) return fail(DVQ_EINVAL, "circuit range not whole Re/Im pairs");
    constexpr int CPW = circuits_per_wave<T, ENT, BVEC>();
    hipLaunchKernelGGL((k_terms_fast<T, NQ, ENT, BVEC>), grid_for(g.total / CPW), dim3(64), lds, s,
                       with_fast_div(g));
    DVQ_CHECK_LAUNCH("k_terms_fast");
    return DVQ_OK;
}

template <typename T, int NQ>
static dvq_status launch_fast(const TermsArgs& g, hipStream_t s) {
    const bool cz = g.ent == DVQ_ENT_CZ_LADDER, bv = g.bkind == DVQ_B_VECTOR;
    if (cz) return bv ? launch_fast_ent<T, NQ, DVQ_ENT_CZ_LADDER, true>(g, s)
                      : launch_fast_ent<T, NQ, DVQ_ENT_CZ_LADDER, false>(g, s);
    return bv ? launch_fast_ent<T, NQ, DVQ_ENT_CNOT_LADDER, true>(g, s)
              : launch_fast_ent<T, NQ, DVQ_ENT_CNOT_LADDER, false>(g, s);
}

// Circuits per wavefront in the prefix-shared form: enough wavefronts to
// cover the chip several times over, chunks of whole Re/Im pairs.
static int64_t shared_chunk(int64_t per_row, int B) {
    const int64_t target_waves = 8192;
    int64_t per_row_waves = (target_waves + B - 1) / B;
    int64_t chunk = (per_row + per_row_waves - 1) / per_row_waves;
    if (chunk < 64) chunk = 64;
    chunk = (chunk + 1) & ~int64_t(1);
    return chunk;
}

template <typename T, int NQ, int ENT, bool BVEC>
static dvq_status launch_shared_ent(const TermsArgs& g, hipStream_t s) {
    const size_t lds = fast_lds_bytes<T, NQ>(g.layers);
    DVQ_TRY_HIP(allow_lds((const void*)k_terms_shared<T, NQ, ENT, BVEC>, lds));
    const int64_t chunk = shared_chunk(g.per_row, g.B);
    const int64_t cpr = (g.per_row + chunk - 1) / chunk;
    hipLaunchKernelGGL((k_terms_shared<T, NQ, ENT, BVEC>), grid_for(cpr * g.B), dim3(64), lds, s, g, chunk,
                       cpr);
    DVQ_CHECK_LAUNCH("k_terms_shared");
    return DVQ_OK;
}

template <typename T, int NQ>
static dvq_status launch_shared(const TermsArgs& g, hipStream_t s) {
    const bool cz = g.ent == DVQ_ENT_CZ_LADDER, bv = g.bkind == DVQ_B_VECTOR;
    if (cz) return bv ? launch_shared_ent<T, NQ, DVQ_ENT_CZ_LADDER, true>(g, s)
                      : launch_shared_ent<T, NQ, DVQ_ENT_CZ_LADDER, false>(g, s);
    return bv ? launch_shared_ent<T, NQ, DVQ_ENT_CNOT_LADDER, true>(g, s)
              : launch_shared_ent<T, NQ, DVQ_ENT_CNOT_LADDER, false>(g, s);
}

// Local cost, or a global-cost range holding beta circuits only (the gamma
// circuits control V(theta), which these kernels do not).
static bool fast_shape(const TermsArgs& g) {
    const bool kind_ok = g.kind == DVQ_COST_LOCAL || g.c0 + g.per_row <= 2 * (int64_t)g.L * g.L;
    return kind_ok && g.n * g.layers <= 1024 && (g.bkind == DVQ_B_PLUS || g.b != nullptr);
}

dvq_status launch_terms_fast(const TermsArgs& g, int precision, hipStream_t s) {
    if (!fast_shape(g)) return DVQ_EUNSUPPORTED;
    if (precision == DVQ_F32) {
        if (g.n == 10) return launch_fast<float, 10>(g, s);
        if (g.n == 11) return launch_fast<float, 11>(g, s);
    } else {
        if (g.n == 10) return launch_fast<double, 10>(g, s);
    }
    return DVQ_EUNSUPPORTED;
}

dvq_status launch_terms_shared(const TermsArgs& g, int precision, hipStream_t s) {
    if (!fast_shape(g)) return DVQ_EUNSUPPORTED;
    if (precision == DVQ_F32) {
        if (g.n == 10) return launch_shared<float, 10>(g, s);
        if (g.n == 11) return launch_shared<float, 11>(g, s);
    } else {
        if (g.n == 10) return launch_shared<double, 10>(g, s);
    }
    return DVQ_EUNSUPPORTED;
}

}  // namespace dvq

// Adjoint gradient with the state in registers: one workgroup of four
// wavefronts per parameter row (n = 10, 11; CZ or CNOT ladder).  Every
// wavefront holds the whole state and runs the register phases (the same
// values, written to the same LDS slots); the Pauli sums are split between
// them.  Same mathematics as k_adjoint (adjoint.hip):
//   x = V(theta)|0>, y = A x (A = sum_l c_l P_l), Psi = <y|y>,
//   local:  u = U_b^dag y, E = sum_k |u_k|^2 (n - 2|k|),
//           v = dC/dE * U_b D u + dC/dPsi * y   (D = diag(n - 2|k|) = sum_j Z_j);
//   global: g = <b|y>, v = dC/dG * g b + dC/dPsi * y;
//   lambda = A^dag v; then the gates are undone on x and lambda together and
//   every RY gives dC/dtheta_k = Re <K_q x_k | lambda_k>.
// The two vectors of the reverse sweep share the registers of one wavefront:
// lanes 0..31 hold x, lanes 32..63 hold lambda (the "half" bit of the
// layouts in wave_state.h), so every undo step is one pass over the
// registers; the inner products pair each lane with lane +- 32 through
// v_permlane32_swap.  Within a layer the RYs commute, so the gradient of each
// RY may be taken before or after undoing the others of the same layer.
// The Pauli sums and U_b are computed on natural-order copies in LDS.
//
// CNOT ladder.  The forward pass leaves the registers in the ladder frame
// (stored index k holds the true amplitude of pi(k), pi the prefix parity;
// wave_state.h).  The reverse sweep mirrors it: x and lambda are loaded in
// that frame (x stored in frame order at the end of the forward pass,
// lambda written in frame order by the Pauli sum), so undoing a layer's
// ladder is a change of interpretation, not of data; the RYs a layer applied
// in the frame are undone in the frame (ladder-paired amplitudes, the lane
// swap for the qubit split between registers and lane bit 0), and each
// layout swap of the forward pass that left the frame is undone by one that
// enters it (relayout_to_ladder).
#include "wave_state.h"

namespace dvq {

// The value lane + 32 holds, in lanes 0..31 (lambda next to x; the upper
// lanes receive the lower half's values, which no caller uses): one
// v_permlane32_swap per 32-bit word.
__device__ __forceinline__ float from_upper(float x) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    return __uint_as_float(r[1]);
}

__device__ __forceinline__ double from_upper(double x) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(x);
    const auto rl = __builtin_amdgcn_permlane32_swap((unsigned)u, (unsigned)u, false, false);
    const auto rh = __builtin_amdgcn_permlane32_swap((unsigned)(u >> 32), (unsigned)(u >> 32), false, false);
    return __longlong_as_double((long long)(((unsigned long long)rh[1] << 32) | rl[1]));
}

// ------------------------------------------------------------ gradient sums
//
// dC/dtheta of the RY on qubit q is Re <K_q x | lambda> with (K x)_0 = -x_1,
// (K x)_1 = x_0 on each amplitude pair of q, i.e. x_0 . lambda_1 - x_1 .
// lambda_0 per pair (a . b = Re(conj(a) b)).  All RYs of one layer commute
// with each other's generators, so the gradients of every qubit a layout
// holds in its registers are taken from the same registers, before any of
// them is undone.  Lambda is brought to the lower lanes once per range and
// chunk (R / CH registers at a time, so at most that many extra registers
// of each component are live); each register r of a chunk then adds, for
// every qubit, lambda at r times x at its pair partner, negated when r is
// the pair's |0> member, with the pair's frame sign.  The W wavefronts of a
// row hold the same registers and take every W-th qubit each.  Each lane
// keeps one partial sum per qubit, written to LDS (gb[q * 33 + lane], lanes
// 0..31);
// flush_grad adds the 32 partials of each qubit once per layer, so no
// cross-lane reduction sits in the sweep's dependency chain.

template <typename T, int R>
constexpr int kGradChunks = (int)sizeof(T) * R > 128 ? 2 : 1;

// Pair structure of qubit Q in layout HI: CZ form (partner r ^ 2^j, lazy
// sign frame when PAR) or ladder frame (partner r ^ 2^j ^ 2^j', j' the
// register bit of Q + 1, sign from the parity of the qubits below Q).
template <int NQ, bool HI, int Q, int PAR, bool LADDER>
struct PairOf {
    using Ly = Lay<NQ, HI>;
    static constexpr int j = Ly::reg(Q);
    static constexpr int jp = (LADDER && Q + 1 < NQ) ? Ly::reg(Q + 1) : -1;
    static_assert(j >= 0 && (!LADDER || Q + 1 == NQ || jp >= 0), "pair not in registers");
    static constexpr int mask = (1 << j) | (jp >= 0 ? (1 << jp) : 0);
    static constexpr int low = !LADDER ? 0 : (HI ? ((1 << (Q - 5)) - 1) : ((1 << Q) - 1));
    static constexpr int partner(int r) { return r ^ mask; }
    static constexpr bool one(int r) { return (r >> j) & 1; }
    static constexpr bool neg(int r) {
        const int r0 = one(r) ? partner(r) : r;
        return LADDER ? odd_bits(r0 & low) : (PAR ? reg_rho<NQ, HI, Q>(r0) : false);
    }
    // the term of register r enters with + (|1> member) or - (|0> member), times the pair sign
    static constexpr bool plus(int r) { return one(r) != neg(r); }
    __device__ static bool lane_neg(int lane) {
        if constexpr (LADDER)
            return HI && (__popc((unsigned)(lane & 31)) & 1);
        else
            return PAR && lane_rho<NQ, HI, Q>(lane);
    }
};

template <typename T, int NQ, bool HI, int PAR, bool LADDER, int W, int Q, int QEND, int C0, int H>
__device__ __forceinline__ void grad_chunk(const T* re, const T* im, const T* lr, const T* li, T* acc, int wave) {
    if constexpr (Q < QEND) {
        if constexpr (Lay<NQ, HI>::reg(Q) >= 0) {
            if (Q % W == wave) {  // each wavefront takes every W-th qubit
                using Pr = PairOf<NQ, HI, Q, PAR, LADDER>;
                T a = acc[Q];
#pragma unroll
                for (int h = 0; h < H; ++h) {
                    const int r = C0 + h, p = Pr::partner(r);
                    a = fmat(Pr::plus(r) ? re[p] : -re[p], lr[h], a);
                    a = fmat(Pr::plus(r) ? im[p] : -im[p], li[h], a);
                }
                acc[Q] = a;
            }
        }
        grad_chunk<T, NQ, HI, PAR, LADDER, W, Q + 1, QEND, C0, H>(re, im, lr, li, acc, wave);
    }
}

// Qubit RB-1 in layout LO, ladder frame: the stored partner of (lane, r) is
// (lane ^ 1, r ^ 2^(RB-1)) and r is the |0> member iff it has even parity.
template <typename T, int NQ, int C0, int H>
__device__ __forceinline__ T grad_lane_chunk(const T* re, const T* im, const T* lr, const T* li, T a) {
    constexpr int j = Lay<NQ, false>::RB - 1;
#pragma unroll
    for (int h = 0; h < H; ++h) {
        const int r = C0 + h, q = r ^ (1 << j);
        if (odd_bits(r)) {
            a = fmat(re[q], lane_xor1(lr[h]), a);
            a = fmat(im[q], lane_xor1(li[h]), a);
        } else {
            a = fmat(-lane_xor1(re[q]), lr[h], a);
            a = fmat(-lane_xor1(im[q]), li[h], a);
        }
    }
    return a;
}

template <typename T, int NQ, bool HI, int PAR, bool LADDER, int W, int Q, int QEND>
__device__ __forceinline__ void grad_store(const T* acc, int lane, double* gb, int wave) {
    if constexpr (Q < QEND) {
        if constexpr (Lay<NQ, HI>::reg(Q) >= 0) {
            using Pr = PairOf<NQ, HI, Q, PAR, LADDER>;
            const T a = Pr::lane_neg(lane) ? -acc[Q] : acc[Q];
            if (lane < 32 && Q % W == wave) gb[Q * 33 + lane] = (double)a;
        }
        grad_store<T, NQ, HI, PAR, LADDER, W, Q + 1, QEND>(acc, lane, gb, wave);
    }
}

// Partial gradient sums of the register qubits [Q, QEND) of layout HI (and,
// with LANEQ, of qubit RB-1 of layout LO in the ladder frame) into gb.
template <typename T, int NQ, bool HI, int PAR, bool LADDER, bool LANEQ, int W, int Q, int QEND>
__device__ __forceinline__ void grad_range(const T* re, const T* im, int lane, double* gb, int wave) {
    constexpr int R = Lay<NQ, HI>::R, CH = kGradChunks<T, R>, H = R / CH;
    constexpr int QL = Lay<NQ, false>::RB - 1;
    T acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = (T)0;
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        T lr[H], li[H];
#pragma unroll
        for (int h = 0; h < H; ++h) {
            lr[h] = from_upper(re[c * H + h]);
            li[h] = from_upper(im[c * H + h]);
        }
        if (c == 0) {
            grad_chunk<T, NQ, HI, PAR, LADDER, W, Q, QEND, 0, H>(re, im, lr, li, acc, wave);
            if constexpr (LANEQ)
                if (QL % W == wave) acc[QL] = grad_lane_chunk<T, NQ, 0, H>(re, im, lr, li, acc[QL]);
        } else {
            grad_chunk<T, NQ, HI, PAR, LADDER, W, Q, QEND, (CH > 1 ? H : 0), H>(re, im, lr, li, acc, wave);
            if constexpr (LANEQ)
                if (QL % W == wave) acc[QL] = grad_lane_chunk<T, NQ, (CH > 1 ? H : 0), H>(re, im, lr, li, acc[QL]);
        }
    }
    grad_store<T, NQ, HI, PAR, LADDER, W, Q, QEND>(acc, lane, gb, wave);
    if constexpr (LANEQ) {
        if (lane < 32 && QL % W == wave) gb[QL * 33 + lane] = (double)acc[QL];
    }
}

// Gradients of the register qubits [Q, QEND), then their RYs undone (CZ form).
template <typename T, int NQ, bool HI, int PAR, int W, int Q, int QEND>
__device__ __forceinline__ void grad_undo_range(T* re, T* im, int lane, const T* trig, int kbase, double* gb,
                                                int wave) {
    grad_range<T, NQ, HI, PAR, false, false, W, Q, QEND>(re, im, lane, gb, wave);
    ry_range<T, NQ, HI, PAR, Q, QEND>(re, im, lane, trig, kbase, (T)-1);
}

template <typename T, int NQ, bool HI, int Q, int QEND>
__device__ __forceinline__ void undo_range_ladder(T* re, T* im, int lane, const T* trig, int kbase) {
    if constexpr (Q < QEND) {
        ry_reg_ladder<T, NQ, HI, Q>(re, im, lane, -trig[2 * (kbase + Q)], -trig[2 * (kbase + Q) + 1]);
        undo_range_ladder<T, NQ, HI, Q + 1, QEND>(re, im, lane, trig, kbase);
    }
}

// Ladder frame: gradients of qubits [Q, QEND) (and of qubit RB-1 across
// lane bit 0 with LANEQ, layout LO), then their RYs undone.
template <typename T, int NQ, bool HI, int W, int Q, int QEND, bool LANEQ = false>
__device__ __forceinline__ void grad_undo_range_ladder(T* re, T* im, int lane, const T* trig, int kbase,
                                                       double* gb, int wave) {
    grad_range<T, NQ, HI, 0, true, LANEQ, W, Q, QEND>(re, im, lane, gb, wave);
    if constexpr (LANEQ) {
        constexpr int k = Lay<NQ, false>::RB - 1;
        ry_lane_ladder_lo<T, NQ>(re, im, -trig[2 * (kbase + k)], -trig[2 * (kbase + k) + 1]);
    }
    undo_range_ladder<T, NQ, HI, Q, QEND>(re, im, lane, trig, kbase);
}

// Sum of the 32 partials of each qubit of the layer into g[0..NQ), by the
// first NQ threads of the block, after a barrier (the partials of every
// wavefront written).  No barrier after it: consecutive layers write
// alternate partial buffers, and a buffer is written again only after the
// next layer's flush barrier, which the reading threads reach once done.
template <int NQ>
__device__ __forceinline__ void flush_grad(const double* gb, double* __restrict__ g, int tid) {
    __syncthreads();
    if (tid < NQ) {
        const double* p = gb + tid * 33;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
        for (int i = 0; i < 32; i += 4) {
            s0 += p[i];
            s1 += p[i + 1];
            s2 += p[i + 2];
            s3 += p[i + 3];
        }
        g[tid] = (s0 + s1) + (s2 + s3);
    }
}

// Layout swap into the ladder frame, the inverse of relayout_ladder: the
// registers (layout FROM_HI, true frame) are written to slot pi^-1(m) of
// their true index m and read back in the other layout in natural slot
// order, so stored index k receives the true amplitude of pi(k).  The lane
// and register parts of pi^-1 overlap in one bit (RB for LO, 5 for HI), so
// each write is one of two per-lane bases plus a compile-time offset.
template <typename T, int NQ, bool FROM_HI>
__device__ __forceinline__ void relayout_to_ladder(T* re, T* im, cplx<T>* S, int lane) {
    using From = Lay<NQ, FROM_HI>;
    constexpr int R = From::R;
    constexpr int SPLIT = FROM_HI ? 5 : From::RB;
    const int ub = ladder_unperm<NQ>(From::glane(lane));
    const int base0 = pad_slot(ub), base1 = pad_slot(ub ^ (1 << SPLIT));
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int u = ladder_unperm<NQ>(From::greg(r));
        const int off = u & ~(1 << SPLIT);
        S[((u >> SPLIT) & 1 ? base1 : base0) + off + (off >> 5)] = {re[r], im[r]};
    }
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

// Lanes 0..31 (half 0), layout LO in the ladder frame, to a natural-order
// region in the true frame: stored k goes to slot pi(k) (two bases by the
// parity of r, as in store_state_ladder).
template <typename T, int NQ>
__device__ __forceinline__ void store_half0_true_lo_ladder(const T* re, const T* im, cplx<T>* S0, int lane) {
    using Lo = Lay<NQ, false>;
    constexpr int R = Lo::R, RB = Lo::RB;
    constexpr int HM = ((1 << NQ) - 1) & ~((1 << RB) - 1);
    if (!(lane & 32)) {
        const int pl = ladder_perm<NQ>(Lo::glane(lane));
        const int base0 = pad_slot(pl), base1 = pad_slot(pl ^ HM);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int off = ladder_perm<NQ>(r) & ((1 << RB) - 1);
            S0[(odd_bits(r) ? base1 : base0) + off + (off >> 5)] = {re[r], im[r]};
        }
    }
    __syncthreads();
}

// H on every register qubit q in [Q, QEND).
template <typename T, int NQ, bool HI, int Q, int QEND>
__device__ __forceinline__ void h_range(T* re, T* im) {
    if constexpr (Q < QEND) {
        constexpr int j = Lay<NQ, HI>::reg(Q);
        if constexpr (j >= 0) {
            constexpr int R = Lay<NQ, HI>::R;
            const T r2 = (T)0.70710678118654752440;
#pragma unroll
            for (int r0 = 0; r0 < R; ++r0) {
                if (r0 & (1 << j)) continue;
                const int r1 = r0 | (1 << j);
                const T ar = re[r0], ai = im[r0], br = re[r1], bi = im[r1];
                re[r0] = (ar + br) * r2;
                im[r0] = (ai + bi) * r2;
                re[r1] = (ar - br) * r2;
                im[r1] = (ai - bi) * r2;
            }
        }
        h_range<T, NQ, HI, Q + 1, QEND>(re, im);
    }
}

// Load both halves from natural-order LDS regions (lanes 0..31 from S0,
// lanes 32..63 from S1) into layout HI / LO, applying S^p.
template <typename T, int NQ, bool HI>
__device__ __forceinline__ void load_halves(T* re, T* im, const cplx<T>* S0, const cplx<T>* S1, int lane,
                                            int p) {
    constexpr int R = Lay<NQ, HI>::R;
    constexpr int N = 1 << NQ;
    const cplx<T>* src = (lane & 32) ? S1 : S0;
    const LadderSign<NQ, HI> ls(lane);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int g = Lay<NQ, HI>::g(lane, r) & (N - 1);
        const cplx<T> v = src[pad_slot(g)];
        const bool flip = p && ls.flip(r);
        re[r] = flip ? -v.re : v.re;
        im[r] = flip ? -v.im : v.im;
    }
    __syncthreads();
}

// Store lanes 0..31 (half 0) into a natural-order region, applying S^p.
template <typename T, int NQ, bool HI>
__device__ __forceinline__ void store_half0(const T* re, const T* im, cplx<T>* S0, int lane, int p) {
    constexpr int R = Lay<NQ, HI>::R;
    if (!(lane & 32)) {
        const LadderSign<NQ, HI> ls(lane);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int g = Lay<NQ, HI>::g(lane, r);
            const bool flip = p && ls.flip(r);
            S0[pad_slot(g)] = flip ? cplx<T>{-re[r], -im[r]} : cplx<T>{re[r], im[r]};
        }
    }
    __syncthreads();
}

// out[k] = sum_l w_l (P_l in)[k] over natural-order regions, w_l = c_l or
// conj(c_l).  (P in)[k] = i^{|x&z|} (-1)^{|z&x|} (-1)^{|z&k|} in[k^x]; with
// k = lane + 64 i the last sign splits into a per-lane part, folded into the
// coefficient once per string, and a per-i part that is uniform over the
// wavefront; the gather address is a per-lane base plus 66 (i ^ (x >> 6)),
// also uniform.
// The W = 4 wavefronts of a row take a quarter of the strings each, for
// every amplitude (a string's own work -- its phase, its uniform offsets --
// is paid by one wavefront, not by all four), into register partial sums;
// the first three write theirs to p0, p1, p2 and the fourth adds them to its
// own, in that order, and writes out.  p0 may be out itself when FRAME is
// off (the fourth wavefront reads and writes the same slot); with FRAME,
// out[k] receives the sum at index pi(k) (the ladder frame: sum index m is
// written to slot pi^-1(m)) and none of p0..p2 may be out.
// A wavefront's strings come from device memory, 64 per vector load (one per
// lane), then one at a time out of the registers (v_readlane); the gathers
// of two strings (n = 10) are issued together before their products.
template <typename T, int NQ, int W, bool FRAME = false>
__device__ __forceinline__ void wave_pauli_sum(cplx<T>* out, const cplx<T>* in, cplx<T>* p0, cplx<T>* p1,
                                               cplx<T>* p2, const dvq_pauli* __restrict__ sp,
                                               const dvq_c128* __restrict__ cp, int L, bool conj_c, int lane,
                                               int wave) {
    static_assert(W == 4, "three partial regions and the last wavefront's registers");
    constexpr int KPL = (1 << NQ) / 64, U = KPL <= 16 ? 2 : 1;  // n = 11: one string at a time (registers)
    const int per = (L + W - 1) / W;
    const int l0 = __builtin_amdgcn_readfirstlane(wave * per < L ? wave * per : L);
    const int l1 = l0 + per < L ? l0 + per : L;
    T ar[KPL], ai[KPL];
#pragma unroll
    for (int i = 0; i < KPL; ++i) ar[i] = ai[i] = (T)0;
    // string (x, z, coefficient): its coefficient with the lane's phase (the
    // uniform power of i by scalar selects, then the lane's sign) and its KPL
    // gathers
    auto fetch = [&](uint32_t x, uint32_t z, double cre, double cim, cplx<T>& c, int& zh, cplx<T>* v) {
        // (a + ib) i^p: p = 1 (-b, a), 2 (-a, -b), 3 (b, -a)
        const int p = (int)__popc(x & z) + 2 * parity(z & x);
        const double a = cre, b = conj_c ? -cim : cim;
        double r = (p & 1) ? b : a, m = (p & 1) ? a : b;
        if (((p + 1) >> 1) & 1) r = -r;
        if (p & 2) m = -m;
        c = {(T)r, (T)m};
        if (parity(z & (uint32_t)lane)) c = {-c.re, -c.im};
        const int bl = lane ^ (int)(x & 63u);
        const cplx<T>* src = in + (bl + (bl >> 5));
        const int xh = (int)(x >> 6);
        zh = (int)(z >> 6);
#pragma unroll
        for (int i = 0; i < KPL; ++i) v[i] = src[66 * (i ^ xh)];
    };
    auto accumulate = [&](const cplx<T>& c, int zh, const cplx<T>* v) {
#pragma unroll
        for (int i = 0; i < KPL; ++i) {
            const bool neg = parity((uint32_t)(zh & i));
            const T cr = neg ? -c.re : c.re, ci = neg ? -c.im : c.im;
            ar[i] = fmat(cr, v[i].re, fmat(-ci, v[i].im, ar[i]));
            ai[i] = fmat(cr, v[i].im, fmat(ci, v[i].re, ai[i]));
        }
    };
    for (int base = l0; base < l1; base += 64) {
        const int nb = l1 - base < 64 ? l1 - base : 64;
        const int j = lane < nb ? base + lane : base;
        const uint32_t lx = sp[j].x, lz = sp[j].z;
        const uint64_t lre = __builtin_bit_cast(uint64_t, cp[j].re), lim = __builtin_bit_cast(uint64_t, cp[j].im);
        auto take = [&](int k, uint32_t& x, uint32_t& z, double& cre, double& cim) {
            x = (uint32_t)__builtin_amdgcn_readlane((int)lx, k);
            z = (uint32_t)__builtin_amdgcn_readlane((int)lz, k);
            cre = __builtin_bit_cast(double, ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(lre >> 32), k) << 32) |
                                                 (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)lre, k));
            cim = __builtin_bit_cast(double, ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(lim >> 32), k) << 32) |
                                                 (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)lim, k));
        };
        int k = 0;
        for (; k + U <= nb; k += U) {
            uint32_t x[U], z[U];
            double cre[U], cim[U];
#pragma unroll
            for (int u = 0; u < U; ++u) take(k + u, x[u], z[u], cre[u], cim[u]);
            cplx<T> c[U], v[U][KPL];
            int zh[U];
#pragma unroll
            for (int u = 0; u < U; ++u) fetch(x[u], z[u], cre[u], cim[u], c[u], zh[u], v[u]);
#pragma unroll
            for (int u = 0; u < U; ++u) accumulate(c[u], zh[u], v[u]);
        }
        for (; k < nb; ++k) {
            uint32_t x, z;
            double cre, cim;
            take(k, x, z, cre, cim);
            cplx<T> c, v[KPL];
            int zh;
            fetch(x, z, cre, cim, c, zh, v);
            accumulate(c, zh, v);
        }
    }
    if (wave < W - 1) {
        cplx<T>* pw = wave == 0 ? p0 : (wave == 1 ? p1 : p2);
#pragma unroll
        for (int i = 0; i < KPL; ++i) pw[pad_slot(lane + 64 * i)] = {ar[i], ai[i]};
    }
    __syncthreads();
    if (wave == W - 1) {
        const int ul = FRAME ? ladder_unperm<NQ>(lane) : 0;
#pragma unroll
        for (int i = 0; i < KPL; ++i) {
            const int k = pad_slot(lane + 64 * i);
            const cplx<T> a = p0[k], b = p1[k], c = p2[k];
            const cplx<T> sum = {((a.re + b.re) + c.re) + ar[i], ((a.im + b.im) + c.im) + ai[i]};
            if constexpr (FRAME)
                out[pad_slot(ul ^ ladder_unperm<NQ>(64 * i))] = sum;
            else
                out[k] = sum;
        }
    }
    __syncthreads();
}

// Householder U_b (= U_b^dagger) applied to a natural-order region in place.
// Every lane reads its amplitudes before the barrier and writes after it, so
// wavefronts that run this redundantly write the same values and never read
// an updated one.
template <typename T, int NQ>
__device__ __forceinline__ void wave_householder(cplx<T>* v, const double* __restrict__ b, int lane) {
    constexpr int N = 1 << NQ, KPL = N / 64;
    const double s = (b[0] > 0.0) ? -1.0 : 1.0;
    double ww = 0.0, dr = 0.0, di = 0.0;
    cplx<T> a[KPL];
#pragma unroll
    for (int i = 0; i < KPL; ++i) {
        const int k = lane + 64 * i;
        const double w = (k == 0 ? 1.0 : 0.0) - s * b[k];
        a[i] = v[pad_slot(k)];
        ww += w * w;
        dr += w * (double)a[i].re;
        di += w * (double)a[i].im;
    }
    ww = wave_sum(ww);
    dr = wave_sum(dr);
    di = wave_sum(di);
    const double fr = 2.0 * dr / ww, fi = 2.0 * di / ww;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < KPL; ++i) {
        const int k = lane + 64 * i;
        const double w = (k == 0 ? 1.0 : 0.0) - s * b[k];
        v[pad_slot(k)] = {(T)(s * ((double)a[i].re - w * fr)), (T)(s * ((double)a[i].im - w * fi))};
    }
    __syncthreads();
}

template <typename T, int NQ, int ENT>
__host__ __device__ constexpr size_t wave_adjoint_lds(int layers, int L) {
    constexpr int N = 1 << NQ;
    constexpr int regions = ENT == DVQ_ENT_CZ_LADDER ? 3 : 4;    // x, y/lambda, v (+ x in the ladder frame)
    return (size_t)(2 * N + (2 * N) / 32) * sizeof(cplx<T>)      // scratch for layout swaps
           + regions * (size_t)(N + N / 32) * sizeof(cplx<T>)
           + (size_t)2 * NQ * 33 * sizeof(double)                // gradient partials, two buffers
           + (size_t)2 * NQ * layers * sizeof(T);                // rotation table
}

template <typename T, int NQ, int ENT, int W>
__global__ void __launch_bounds__(64 * W)
k_adjoint_wave(const double* __restrict__ theta, int layers, const dvq_c128* __restrict__ coeffs,
               const dvq_pauli* __restrict__ strings, int L, int per_row_system, int bkind,
               const double* __restrict__ bvec, int kind, double* __restrict__ Cout,
               double* __restrict__ grad) {
    constexpr int N = 1 << NQ;
    constexpr int R = Lay<NQ, false>::R;
    constexpr int N1 = N + N / 32;
    extern __shared__ __align__(16) unsigned char smem[];
    cplx<T>* S = reinterpret_cast<cplx<T>*>(smem);
    cplx<T>* RX = S + (2 * N + (2 * N) / 32);
    cplx<T>* RY = RX + N1;
    cplx<T>* RV = RY + N1;
    constexpr bool CNOT = ENT == DVQ_ENT_CNOT_LADDER;
    cplx<T>* RXF = RV + N1;  // x in the ladder frame (CNOT ladder only)
    double* gb = reinterpret_cast<double*>(CNOT ? RXF + N1 : RV + N1);  // gradient partials [2][NQ][33]
    T* trig = reinterpret_cast<T*>(gb + 2 * NQ * 33);
    // W wavefronts per row: each runs the register phases redundantly (same
    // values written to the same LDS slots, every hand-over fenced by a
    // barrier) and takes 1/W of the Pauli sums; wavefront 0 writes the results.
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t row = blockIdx.x;
    const int P = NQ * layers;
    const int64_t sys = per_row_system ? row * L : 0;
    const dvq_pauli* __restrict__ sp = strings + sys;
    const dvq_c128* __restrict__ cp = coeffs + sys;
    rotation_table<T>(theta + row * P, P, trig, lane);  // ends with a barrier

    // forward: both halves start in |0> and evolve identically
    T re[R], im[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        re[r] = (r == 0 && (lane & 31) == 0) ? (T)1 : (T)0;
        im[r] = (T)0;
    }
    const int pf = layers & 1;
    if constexpr (!CNOT) {
        forward_layers<T, NQ>(re, im, S, trig, layers, lane);
        if (pf)
            store_half0<T, NQ, true>(re, im, RX, lane, 1);
        else
            store_half0<T, NQ, false>(re, im, RX, lane, 0);
    } else {
        // ends in the ladder frame, layout HI for an odd layer count
        forward_layers_ladder<T, NQ>(re, im, S, trig, layers, lane);
        if (pf) {
            store_half0<T, NQ, true>(re, im, RXF, lane, 0);
            relayout_ladder<T, NQ, true>(re, im, S, lane);  // -> LO, true frame
            store_half0<T, NQ, false>(re, im, RX, lane, 0);
        } else {
            store_half0<T, NQ, false>(re, im, RXF, lane, 0);
            store_half0_true_lo_ladder<T, NQ>(re, im, RX, lane);
        }
    }

    // y = A x, Psi = <y|y>
    wave_pauli_sum<T, NQ, W>(RY, RX, RY, RV, S, sp, cp, L, false, lane, wave);  // RV, S free until later
    double ps = 0.0;
    for (int k = lane; k < N; k += 64) {
        const cplx<T> a = RY[pad_slot(k)];
        ps += (double)a.re * a.re + (double)a.im * a.im;
    }
    const double Psi = wave_sum(ps);

    double cost;
    if (kind == DVQ_COST_LOCAL) {
        double aE, aPsi;
        if (bkind == DVQ_B_PLUS) {
            // U_b = H^n and H Z_j H = X_j: E = <y|H^n D H^n|y> = sum_j <y|X_j|y>
            // and H^n D H^n y = sum_j X_j y (D = sum_j Z_j), n bit-flip
            // gathers per amplitude with the amplitudes split between the W
            // wavefronts (E summed in float64 from the products)
            constexpr int KW = (N / 64) / W;
            double es = 0.0;
#pragma unroll
            for (int i = 0; i < KW; ++i) {
                const int k = lane + 64 * (wave * KW + i);
                const cplx<T> yk = RY[pad_slot(k)];
                T sr = (T)0, si = (T)0;
#pragma unroll
                for (int j = 0; j < NQ; ++j) {
                    const cplx<T> yj = RY[pad_slot(k ^ (1 << j))];
                    sr += yj.re;
                    si += yj.im;
                    es += (double)yk.re * yj.re + (double)yk.im * yj.im;
                }
                RV[pad_slot(k)] = {sr, si};
            }
            es = wave_sum(es);
            if (lane == 0) gb[wave] = es;  // gb holds the gradient partials only from the reverse sweep on
            __syncthreads();
            double E = 0.0;
            for (int v = 0; v < W; ++v) E += gb[v];
            cost = 0.5 - 0.5 * E / (NQ * Psi);
            aE = -0.5 / (NQ * Psi);
            aPsi = 0.5 * E / (NQ * Psi * Psi);
        } else {
            for (int k = lane; k < N; k += 64) RV[pad_slot(k)] = RY[pad_slot(k)];
            __syncthreads();
            wave_householder<T, NQ>(RV, bvec, lane);
            double es = 0.0;
            cplx<T> a[N / 64];
#pragma unroll
            for (int i = 0; i < N / 64; ++i) {
                const int k = lane + 64 * i;
                a[i] = RV[pad_slot(k)];
                es += ((double)a[i].re * a[i].re + (double)a[i].im * a[i].im) *
                      (double)(NQ - 2 * (int)__popc((unsigned)k));
            }
            __syncthreads();  // read by every wavefront before the update
#pragma unroll
            for (int i = 0; i < N / 64; ++i) {
                const int k = lane + 64 * i;
                const T d = (T)(NQ - 2 * (int)__popc((unsigned)k));
                RV[pad_slot(k)] = {a[i].re * d, a[i].im * d};
            }
            const double E = wave_sum(es);
            __syncthreads();
            cost = 0.5 - 0.5 * E / (NQ * Psi);
            aE = -0.5 / (NQ * Psi);
            aPsi = 0.5 * E / (NQ * Psi * Psi);
            wave_householder<T, NQ>(RV, bvec, lane);
        }
        cplx<T> w[N / 64];
#pragma unroll
        for (int i = 0; i < N / 64; ++i) w[i] = RV[pad_slot(lane + 64 * i)];
        __syncthreads();  // read by every wavefront before the update
#pragma unroll
        for (int i = 0; i < N / 64; ++i) {
            const int k = lane + 64 * i;
            const cplx<T> y = RY[pad_slot(k)];
            RV[pad_slot(k)] = {(T)(aE * w[i].re + aPsi * y.re), (T)(aE * w[i].im + aPsi * y.im)};
        }
        __syncthreads();
    } else {
        const double invs = 1.0 / sqrt((double)N);
        double gr = 0.0, gi = 0.0;
        for (int k = lane; k < N; k += 64) {
            const double bk = bkind == DVQ_B_PLUS ? invs : bvec[k];
            const cplx<T> y = RY[pad_slot(k)];
            gr += bk * y.re;
            gi += bk * y.im;
        }
        gr = wave_sum(gr);
        gi = wave_sum(gi);
        const double G = gr * gr + gi * gi;
        cost = 1.0 - G / Psi;
        const double aG = -1.0 / Psi, aPsi = G / (Psi * Psi);
        for (int k = lane; k < N; k += 64) {
            const double bk = bkind == DVQ_B_PLUS ? invs : bvec[k];
            const cplx<T> y = RY[pad_slot(k)];
            RV[pad_slot(k)] = {(T)(aG * gr * bk + aPsi * y.re), (T)(aG * gi * bk + aPsi * y.im)};
        }
        __syncthreads();
    }
    // lambda = A^dag v -> RY (in the ladder frame for the CNOT ladder)
    // partials: y (RY) and the swap scratch S are dead; with the ladder frame
    // the output is permuted, so the first partial goes to RX (the reverse
    // sweep reads x from RXF)
    wave_pauli_sum<T, NQ, W, CNOT>(RY, RV, CNOT ? RX : RY, S, S + N1, sp, cp, L, true, lane, wave);

    // reverse sweep: x in lanes 0..31, lambda in lanes 32..63
    double* g = grad + row * P;
    // layer l's partials go to buffer l mod 2 (see flush_grad)
    auto gbl = [&](int l) { return gb + (l & 1) * NQ * 33; };
    if constexpr (CNOT) {
        constexpr int RB = Lay<NQ, false>::RB;
        if (pf)
            load_halves<T, NQ, true>(re, im, RXF, RY, lane, 0);
        else
            load_halves<T, NQ, false>(re, im, RXF, RY, lane, 0);
        for (int l = layers - 1; l >= 1; --l) {
            const int kb = l * NQ;
            if (l & 1) {
                // odd layer (forward: HI qubits in the frame, swap to LO,
                // LO qubits 0..4): starts in LO, true state of its RYs
                grad_undo_range<T, NQ, false, 0, W, 0, 5>(re, im, lane, trig, kb, gbl(l), wave);
                relayout_to_ladder<T, NQ, false>(re, im, S, lane);
                grad_undo_range_ladder<T, NQ, true, W, 5, NQ>(re, im, lane, trig, kb, gbl(l), wave);
            } else {
                // even layer >= 2 (forward: LO qubits 0..RB-1 in the frame,
                // swap to HI, HI qubits 5..NQ-1): starts in HI
                grad_undo_range<T, NQ, true, 0, W, 5, NQ>(re, im, lane, trig, kb, gbl(l), wave);
                relayout_to_ladder<T, NQ, true>(re, im, S, lane);
                // qubit RB-1 across lane bit 0 when it is below 5 (else in HI above)
                grad_undo_range_ladder<T, NQ, false, W, 0, RB - 1, (RB - 1 < 5)>(re, im, lane, trig, kb, gbl(l), wave);
            }
            flush_grad<NQ>(gbl(l), g + kb, threadIdx.x);
        }
        // layer 0 (forward: LO qubits, plain swap, HI qubits RB..NQ-1): starts in HI
        grad_undo_range<T, NQ, true, 0, W, RB, NQ>(re, im, lane, trig, 0, gbl(0), wave);
        relayout<T, NQ, true>(re, im, S, lane);
        grad_undo_range<T, NQ, false, 0, W, 0, NQ>(re, im, lane, trig, 0, gbl(0), wave);
        flush_grad<NQ>(gbl(0), g, threadIdx.x);
        if (threadIdx.x == 0) Cout[row] = cost;
        return;
    }
    int l = layers - 1;
    if (pf) {
        // last layer even-indexed: ended in HI with p = 1 after its ladder
        load_halves<T, NQ, true>(re, im, RX, RY, lane, 1);
        grad_undo_range<T, NQ, true, 0, W, Lay<NQ, false>::RB, NQ>(re, im, lane, trig, l * NQ, gbl(l), wave);
        relayout<T, NQ, true>(re, im, S, lane);
        grad_undo_range<T, NQ, false, 0, W, 0, NQ>(re, im, lane, trig, l * NQ, gbl(l), wave);
        flush_grad<NQ>(gbl(l), g + l * NQ, threadIdx.x);
        --l;
    } else {
        load_halves<T, NQ, false>(re, im, RX, RY, lane, 0);
    }
    for (; l >= 1; l -= 2) {
        // odd layer l (p = 1 during its RYs): LO qubits 0..4, swap, HI qubits
        grad_undo_range<T, NQ, false, 1, W, 0, 5>(re, im, lane, trig, l * NQ, gbl(l), wave);
        relayout<T, NQ, false>(re, im, S, lane);
        grad_undo_range<T, NQ, true, 1, W, 0, NQ>(re, im, lane, trig, l * NQ, gbl(l), wave);
        flush_grad<NQ>(gbl(l), g + l * NQ, threadIdx.x);
        // even layer l - 1 (p = 0): HI qubits RB..NQ-1, swap, LO qubits
        grad_undo_range<T, NQ, true, 0, W, Lay<NQ, false>::RB, NQ>(re, im, lane, trig, (l - 1) * NQ, gbl(l - 1), wave);
        relayout<T, NQ, true>(re, im, S, lane);
        grad_undo_range<T, NQ, false, 0, W, 0, NQ>(re, im, lane, trig, (l - 1) * NQ, gbl(l - 1), wave);
        flush_grad<NQ>(gbl(l - 1), g + (l - 1) * NQ, threadIdx.x);
    }
    if (threadIdx.x == 0) Cout[row] = cost;
}

// Wavefronts per row.  Four (one per SIMD of the row's CU) beat one at
// every batch size measured (1 to 4096 rows, n = 10, 8 layers, L = 64): the
// Pauli sums split four ways, the register phases run alongside, and a
// row's LDS holds a CU to two workgroups, so one wavefront per row would
// leave two of the four SIMDs idle.
constexpr int kRowWaves = 4;

template <typename T, int NQ, int ENT, int W>
static dvq_status launch_adjoint_wave_w(const dvq_ansatz* an, const double* theta, int B, const dvq_c128* coeffs,
                                        const dvq_pauli* strings, int L, int per_row_system, int bkind,
                                        const double* b, int kind, double* C, double* grad, hipStream_t s) {
    const size_t lds = wave_adjoint_lds<T, NQ, ENT>(an->layers, L);
    if (lds > kMaxLdsBytes) return DVQ_EUNSUPPORTED;
    DVQ_TRY_HIP(allow_lds((const void*)k_adjoint_wave<T, NQ, ENT, W>, lds));
    hipLaunchKernelGGL((k_adjoint_wave<T, NQ, ENT, W>), dim3(B), dim3(64 * W), lds, s, theta, an->layers, coeffs,
                       strings, L, per_row_system, bkind, b, kind, C, grad);
    DVQ_CHECK_LAUNCH("k_adjoint_wave");
    return DVQ_OK;
}

template <typename T, int NQ, int ENT>
static dvq_status launch_adjoint_wave_ent(const dvq_ansatz* an, const double* theta, int B,
                                          const dvq_c128* coeffs, const dvq_pauli* strings, int L,
                                          int per_row_system, int bkind, const double* b, int kind,
                                          double* C, double* grad, hipStream_t s) {
    return launch_adjoint_wave_w<T, NQ, ENT, kRowWaves>(an, theta, B, coeffs, strings, L, per_row_system, bkind,
                                                        b, kind, C, grad, s);
}

template <typename T, int NQ>
static dvq_status launch_adjoint_wave(const dvq_ansatz* an, const double* theta, int B,
                                      const dvq_c128* coeffs, const dvq_pauli* strings, int L,
                                      int per_row_system, int bkind, const double* b, int kind,
                                      double* C, double* grad, hipStream_t s) {
    if (an->entangler == DVQ_ENT_CZ_LADDER)
        return launch_adjoint_wave_ent<T, NQ, DVQ_ENT_CZ_LADDER>(an, theta, B, coeffs, strings, L, per_row_system,
                                                                 bkind, b, kind, C, grad, s);
    return launch_adjoint_wave_ent<T, NQ, DVQ_ENT_CNOT_LADDER>(an, theta, B, coeffs, strings, L, per_row_system,
                                                               bkind, b, kind, C, grad, s);
}

// Dispatch for the register-resident adjoint; DVQ_EUNSUPPORTED when the
// shape has no such kernel (the LDS kernel then runs).
dvq_status launch_adjoint_fast(const dvq_ansatz* an, const double* theta, int B, int precision,
                               const dvq_c128* coeffs, const dvq_pauli* strings, int L,
                               int per_row_system, int bkind, const double* b, int kind, double* C,
                               double* grad, hipStream_t s) {
    if (an->n * an->layers > 1024) return DVQ_EUNSUPPORTED;
    if (precision == DVQ_F32) {
        if (an->n == 10)
            return launch_adjoint_wave<float, 10>(an, theta, B, coeffs, strings, L, per_row_system, bkind, b,
                                                  kind, C, grad, s);
        if (an->n == 11)
            return launch_adjoint_wave<float, 11>(an, theta, B, coeffs, strings, L, per_row_system, bkind, b,
                                                  kind, C, grad, s);
    } else if (an->n == 10) {
        return launch_adjoint_wave<double, 10>(an, theta, B, coeffs, strings, L, per_row_system, bkind, b,
                                               kind, C, grad, s);
    }
    return DVQ_EUNSUPPORTED;
}

}  // namespace dvq
